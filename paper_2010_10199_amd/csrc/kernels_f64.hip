// FP64 instantiation of the transform kernels and launchers.
#include "kernels_impl.h"

namespace gt {
template int launch_forward<double>(gt_plan *, const void *, const double *, void *, hipStream_t);
template int launch_adjoint<double>(gt_plan *, const void *, const double *, void *, hipStream_t);
template int launch_node_grad<double>(gt_plan *, const void *, const void *, void *, hipStream_t);
template int launch_prepare_nodes<double>(gt_plan *, const void *, hipStream_t);
}  // namespace gt
