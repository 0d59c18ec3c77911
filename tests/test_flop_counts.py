"""The FLOP constants the benchmark uses for its roofline equal the oracle's
own count (counting scalar), so the two cannot drift apart."""
import bench


def test_bench_flop_constants_match_oracle(orc):
    from oracle import count_flops
    t = count_flops.table()
    for d in ("x", "y"):
        ref = t[f"euler_2d_{d}"]
        got = bench.FLOPS_2D[d]
        assert abs(got["interface"] - ref["interface"]) < 0.5
        assert abs(got["cell_flux"] - ref["cell_flux"]) < 0.5
        assert got["cell_update"] == ref["cell_update"]


def test_bench_order_flop_constants_match_oracle(orc):
    from oracle import count_flops
    t = count_flops.table()
    for r, v in bench.FLOPS_2D_ORDER_IR.items():
        key = "euler_2d_x" if r == 3 else f"euler_2d_r{r}_x"
        assert abs(v - t[key]["interface"]) < 0.5, (r, v, t[key])
