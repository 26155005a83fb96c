"""Host-side logic of the benchmark that needs no GPU: the HBM bytes a timing record takes from
the counter table for the launch forms the tuner chose."""
import bench

KH = "0123456789abcdef"


def table():
    def e(b):
        return {"bytes_per_launch": b}
    return {"kernels": {
        "gather_12": {"kernel_hash": KH, "forms": {
            "gt::k_fwd_gather2<float, 6, 0, 0>": e(1), "gt::k_fwd_gather2<float, 6, 0, 1>": e(2),
            "gt::k_fwd_gather2<float, 6, 0, 2>": e(3), "gt::k_fwd_gather2<float, 6, 1, 0>": e(4),
            "gt::k_fwd_gather2<float, 6, 1, 1>": e(5), "gt::k_fwd_gather2<float, 6, 1, 2>": e(6)}},
        "pack_fwd_12": {"kernel_hash": KH, "forms": {
            "gt::k_fwd_pack2<float, 0>": e(7), "gt::k_fwd_pack2<float, 6>": e(8)}},
        "gather_2d": {"kernel_hash": KH, "forms": {
            "gt::k_gather_cell<float, 2, 6>": e(9), "gt::k_gather_poly2<float>": e(10),
            "gt::k_gather_sorted<float, 2, 6>": e(11)}},
        "pack_fwd_2d": {"kernel_hash": KH, "forms": {
            "gt::k_pack_fwd<float, 2>": e(12), "gt::k_pack_poly2<6>": e(13)}},
        "empty_adj": {"kernel_hash": KH, "forms": {
            "gt::k_empty_adj<float>": e(14), "gt::k_empty_part<float>": e(15)}},
        "spread_12": {"kernel_hash": KH, "forms": {"gt::k_adj_spread2<float, 6>": e(16)},
                      "bytes_per_launch": 16},
    }}


def tuning(f1, f2):
    return {"gather": {"1": {"chosen": f1}, "2": {"chosen": f2}}}


def test_shared_gather_takes_the_chosen_pair_of_forms():
    code = {"sorted": 0, "cell": 1, "poly": 2}
    for f1 in ("sorted", "cell"):
        for f2 in ("sorted", "cell", "poly"):
            got = bench.counted_bytes(table(), "gather_12", tuning(f1, f2), KH)
            assert got == 1 + 3 * code[f1] + code[f2]


def test_shared_pack_follows_the_order_2_form():
    assert bench.counted_bytes(table(), "pack_fwd_12", tuning("cell", "poly"), KH) == 8
    assert bench.counted_bytes(table(), "pack_fwd_12", tuning("cell", "cell"), KH) == 7
    assert bench.counted_bytes(table(), "pack_fwd_12", tuning("sorted", "sorted"), KH) == 7


def test_separate_records_and_summed_records():
    assert bench.counted_bytes(table(), "gather_2d", tuning("cell", "poly"), KH) == 10
    assert bench.counted_bytes(table(), "gather_2d", tuning("cell", "sorted"), KH) == 11
    assert bench.counted_bytes(table(), "pack_fwd_2d", tuning("cell", "poly"), KH) == 13
    assert bench.counted_bytes(table(), "pack_fwd_2d", tuning("cell", "cell"), KH) == 12
    assert bench.counted_bytes(table(), "empty_adj", tuning("cell", "cell"), KH) == 29
    assert bench.counted_bytes(table(), "spread_12", tuning("cell", "cell"), KH) == 16


def test_other_sources_or_missing_forms_give_none():
    assert bench.counted_bytes(table(), "gather_12", tuning("cell", "poly"), "ffffffffffffffff") is None
    t = table()
    del t["kernels"]["gather_12"]["forms"]["gt::k_fwd_gather2<float, 6, 1, 2>"]
    assert bench.counted_bytes(t, "gather_12", tuning("cell", "poly"), KH) is None
    assert bench.counted_bytes(table(), "gather_12", {"gather": {"1": {"chosen": "direct"}}}, KH) is None
    assert bench.counted_bytes(table(), "no_such_record", tuning("cell", "poly"), KH) is None
