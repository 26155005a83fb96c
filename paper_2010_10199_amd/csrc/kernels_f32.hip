// FP32 instantiation of the transform kernels and launchers.
#include "kernels_impl.h"

namespace gt {
template int launch_forward<float>(gt_plan *, const void *, const float *, void *, hipStream_t);
template int launch_adjoint<float>(gt_plan *, const void *, const float *, void *, hipStream_t);
template int launch_node_grad<float>(gt_plan *, const void *, const void *, void *, hipStream_t);
template int launch_prepare_nodes<float>(gt_plan *, const void *, hipStream_t);
}  // namespace gt
