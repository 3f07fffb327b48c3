"""The benchmark's roofline arithmetic (CPU): per-child ops and bytes and the
side of the ridge point each order falls on."""
import bench


def test_ops_and_bytes_per_child():
    # SQ at m = 20: C(19, 2) = 171 column pairs, one xor, one popcount and one
    # multiply-add each
    assert bench.ops_per_eval(20, 0) == 171 * 3
    # the winner's 80-byte row and two 4-byte keys read; the row and its key written
    assert bench.child_bytes(20) == (88, 84)
    assert bench.child_bytes(36) == (36 * 2 * 4 + 8, 36 * 2 * 4 + 4)
    assert bench.child_bytes(100) == (100 * 4 * 4 + 8, 100 * 4 * 4 + 4)


def test_ridge_point_sides():
    """Up to m = 40 the children kernel is on the HBM side of the ridge point
    of the SQ mix peak over 8 TB/s, from m = 44 on the ALU side."""
    def side(m):
        rd, wr = bench.child_bytes(m)
        intensity = bench.ops_per_eval(m, 0) / (rd + wr)
        ridge = bench.alu_peak_tops(m, 0) * 1e12 / (bench.HBM_PEAK_GBS * 1e9)
        return "hbm" if intensity < ridge else "alu"
    assert [side(m) for m in (8, 20, 32, 36, 40)] == ["hbm"] * 5
    assert [side(m) for m in (44, 64, 100, 128)] == ["alu"] * 4
    assert abs(bench.alu_peak_tops(20, 0) - 47.19) < 0.01
