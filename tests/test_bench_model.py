"""The work model of the benchmark (CPU): the algorithmic flop counts per cell
and step of the fused ADER-DG step reproduce the table of per-degree counts
derived from the Kronecker-factored operators (N+1 Picard sweeps, Euler flux
12 flops, Rusanov 48, signal speed 8), and the FV model is monotone in the
measured work."""

import bench

# flops per cell-step for N = 1..9 with I = N+1 sweeps (predictor, corrector, CFL)
TABLE = {1: 738, 2: 2299, 3: 5708, 4: 12117, 5: 22966, 6: 39983, 7: 65184, 8: 100873, 9: 149642}


def test_dg_flop_model_matches_the_per_degree_table():
    for N, want in TABLE.items():
        pred, rest = bench.dg_flops_per_cell(N, 3, N + 1)
        assert abs(pred + rest - want) <= 1, (N, pred + rest, want)


def test_dg_flop_model_terms():
    N, M = 5, 3
    n = N + 1
    pred1, rest = bench.dg_flops_per_cell(N, M, 1)
    # one sweep: fluxes at n^2 nodes, two n x n contractions over n*M columns
    # per time/space line, the update and the convergence check
    assert pred1 == n * n * 12 + 2 * (2 * n ** 3 * M) + 2 * (2 * n * n * M)
    pred0, rest0 = bench.dg_flops_per_cell(N, M, 0)
    assert pred0 == 0 and rest0 == rest


def test_fv_flop_model_grows_with_the_measured_work():
    base = bench.fv_flops_per_cell(4, 3, 1.0, 1.0)
    assert bench.fv_flops_per_cell(4, 3, 2.0, 1.0) > base
    assert bench.fv_flops_per_cell(4, 3, 1.0, 2.0) > base
    # the kappa~ application (2 n^3 M = 750 flops at n = 5) dominates its term
    d = bench.fv_flops_per_cell(4, 3, 1.0, 2.0) - base
    assert 750 < d < 2000


def test_dg2d_flop_model_values():
    """Regression values of the 2-D flop model at N = 5 (one sweep per cell)."""
    pred, rest = bench.dg2d_flops_per_cell(5, 1.0)
    assert pred == 2 * 216 * 18 + 6 * 1296 * 4 + 4 * 216 * 4 == 42336
    assert rest == 21744 + 17556


def test_dg3d_flop_model_values():
    """Regression values of the 3-D flop model at N = 3 (one sweep per cell)."""
    pred, rest = bench.dg3d_flops_per_cell(3, 1.0)
    assert pred == 3 * 256 * 23 + 8 * 1024 * 5 + 5 * 256 * 5 == 65024
    assert rest > 0


def test_roofline_bound_is_hbm_at_n1_and_alu_at_n5():
    """The fused step's time bound: algorithmic bytes (2 n M 8 per cell) at
    8 TB/s against algorithmic flops at the FP64 VALU peak; N = 1 sits below
    the ridge point (about 7.7 flop/B against 9.8), N = 5 far above."""
    C, K = 100_000, 10
    lo = bench.roofline_entry(1, C, 3, K, 1e-3, 2 * C * K, "fp64")
    assert lo["bound"] == "hbm" and lo["unit"] == "GB/s"
    assert lo["algorithmic_bytes_per_launch"] == 2 * 2 * 3 * 8 * C
    hi = bench.roofline_entry(5, C, 3, K, 1e-3, 6 * C * K, "fp64")
    assert hi["bound"] == "alu" and hi["peak"] == bench.PEAK_FP64_VALU
    assert abs(hi["frac"] - hi["achieved"] / hi["peak"]) <= 1e-3
