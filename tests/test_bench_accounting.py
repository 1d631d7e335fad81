"""Host-side checks of the bench's flop accounting: the per-slice product
counts follow the kernels' polynomial and squaring loops, and the three-product
form is counted only where the kernels use it."""
import numpy as np

import bench


def _products_adjoint(s, q, qb, keep_x2, sampled=False):
    # W = bloc xprev^dag: one product.  Block polynomial by Paterson-Stockmeyer
    # in M^2: three products for M^2 (two when the expm kept X^2, which it
    # forms when q >= 2); the digits above the first one that needs a product
    # are folded in for free (one digit when qb is odd, two when even); three
    # per remaining digit; the last step two, plus the top-left block when
    # squarings follow; each squaring three, the last without the top-left
    # block.
    n = 1 + (2 if keep_x2 and q >= 2 else 3)
    top = (qb - 2) // 2
    t = top - 1 if qb % 2 else (top - 2 if top > 0 else -1)
    while t >= 0:
        n += 3
        t -= 1
    if sampled and s == 0:
        return n  # the last step's entries on the vector ALU
    n += 2 + (1 if s > 0 else 0)
    for j in range(s):
        n += 2 + (1 if j + 1 < s else 0)
    return n


def _products_expm(s, q, ps):
    # Horner: one product per step from degree q down to 1.  Paterson-Stockmeyer
    # in X^2: X^2, then (q >= 3) one per digit below the folded top ones and
    # the last step.  Then one per squaring.
    n = 0
    if q >= 2 and not ps:
        n = q - 1
    elif q >= 2:
        n = 1
        if q >= 3:
            top = (q - 2) // 2
            t = top - 1 if q % 2 else top - 2
            while t >= 0:
                n += 1
                t -= 1
            n += 1
    return n + s


def test_adjoint_product_count_matches_the_loop_structure():
    for s in range(0, 4):
        for qb in range(2, 10):
            q = max(qb - 1, 1)
            plan = np.array([[s, q, qb]], dtype=np.int32)
            for prec, keep in (("fp32", True), ("fp64", False), ("bf16x3", False)):
                f = bench.slice_flops(plan, 64, 12, prec)
                assert f["adjoint_8d3"] == 8.0 * 64 ** 3 * _products_adjoint(s, q, qb, keep)
            f = bench.slice_flops(plan, 16, 8, "fp32")  # d = 16 keeps no X^2
            assert f["adjoint_8d3"] == 8.0 * 16 ** 3 * _products_adjoint(s, q, qb, False)


def test_sampled_last_step_is_counted_where_it_runs():
    from workloads import make_config

    runs = bench.permutation_runs(make_config(3, N=4).Hc)
    assert runs == 6  # X_i and Y_i share their columns: two runs per group of four
    for s in range(0, 3):
        for qb in range(2, 9):
            q = max(qb - 1, 1)
            plan = np.array([[s, q, qb]], dtype=np.int32)
            f = bench.slice_flops(plan, 64, 12, "fp32", runs)
            assert f["adjoint_8d3"] == 8.0 * 64 ** 3 * _products_adjoint(s, q, qb, True, True)
            assert f["adjoint_valu"] == (16.0 * 64 * 64 * runs if s == 0 else 0.0)
            # also at d = 128 with at most 16 controls
            g = bench.slice_flops(plan, 128, 14, "fp32", runs)
            assert g["adjoint_8d3"] == 8.0 * 128 ** 3 * _products_adjoint(s, q, qb, True, True)
            # not at d = 16, nor at d = 128 with more controls, nor in FP64 or split BF16
            for d, mm, prec, keep in ((16, 12, "fp32", False), (128, 17, "fp32", True), (64, 12, "fp64", False),
                                      (64, 12, "bf16x3", False)):
                g = bench.slice_flops(plan, d, mm, prec, runs)
                assert g["adjoint_8d3"] == 8.0 * d ** 3 * _products_adjoint(s, q, qb, keep) and g["adjoint_valu"] == 0


def test_permutation_runs():
    from workloads import make_config, random_hermitian

    assert bench.permutation_runs(make_config(2, N=4).Hc) == 4
    assert bench.permutation_runs(make_config(4, N=4).Hc) == 7  # 14 controls, the last group X_6 and Y_6
    rng = np.random.default_rng(3)
    assert bench.permutation_runs(np.stack([random_hermitian(8, rng)])) is None
    H = np.zeros((4, 4), dtype=np.complex128)
    H[0, 1] = H[1, 0] = H[2, 2] = 1.0  # row 3 empty: a permutation with an empty row
    assert bench.permutation_runs(np.stack([H, 2 * H])) == 1
    H2 = H.copy()
    H2[3, 1] = 1.0  # column 1 hit twice
    assert bench.permutation_runs(np.stack([H2])) is None


def test_expm_product_count_matches_the_loop_structure():
    for s in range(0, 4):
        for q in range(1, 12):
            plan = np.array([[s, q, q + 1]], dtype=np.int32)
            for d, prec, ps in ((64, "fp32", False), (64, "fp64", False), (128, "fp32", True), (128, "fp64", False)):
                f = bench.slice_flops(plan, d, 12, prec)
                g = 6.0 if (d <= 64 or prec == "fp32") else 8.0
                assert f["expm"] == g * d ** 3 * _products_expm(s, q, ps), (d, prec, s, q)


def test_three_product_form_is_counted_where_used():
    plan = np.array([[0, 3, 4], [1, 3, 4]], dtype=np.int32)
    d = 64
    f32 = bench.slice_flops(plan, d, 12, "fp32")
    f64 = bench.slice_flops(plan, d, 12, "fp64")
    b16 = bench.slice_flops(plan, d, 12, "bf16x3")
    n_adj, n_adj_keep = 6 + 9, 5 + 8
    assert f32["adjoint"] == 6.0 * d ** 3 * n_adj_keep and f64["adjoint"] == 6.0 * d ** 3 * n_adj
    assert b16["adjoint"] == 24.0 * d ** 3 * n_adj and b16["adjoint_8d3"] == 8.0 * d ** 3 * n_adj
    # expm: q - 1 + s products; scans: one per direction; all three-product
    assert f32["expm"] == 6.0 * d ** 3 * (2 + 3) and f64["expm"] == 6.0 * d ** 3 * (2 + 3)
    assert f32["scan"] == 2 * 6.0 * d ** 3 * 2 and f64["scan"] == 2 * 6.0 * d ** 3 * 2
    # split BF16: FP32 three-product expm and scans
    assert b16["scan"] == f32["scan"] and b16["expm"] == f32["expm"]
    # d = 16 uses the four-product form everywhere; at d = 128 the FP32 expm
    # and adjoint use the three-product form and FP64 does not
    f = bench.slice_flops(plan, 16, 8, "fp32")
    assert f["adjoint"] == f["adjoint_8d3"] == 8.0 * 16 ** 3 * n_adj and f["expm"] == 8.0 * 16 ** 3 * 5
    f = bench.slice_flops(plan, 128, 14, "fp32")
    assert f["adjoint"] == 6.0 * 128 ** 3 * n_adj_keep and f["expm"] == 6.0 * 128 ** 3 * 5
    assert f["scan"] == 2 * 8.0 * 128 ** 3 * 2
    f = bench.slice_flops(plan, 128, 14, "fp64")
    assert f["adjoint"] == f["adjoint_8d3"] == 8.0 * 128 ** 3 * n_adj and f["expm"] == 8.0 * 128 ** 3 * 5


def test_more_than_one_gpu_is_refused():
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
    assert '"metric"' not in r.stdout


def test_gradient_error_is_taken_per_problem():
    """A small-gradient problem's error counts against its own scale, not the
    batch's largest gradient."""
    import torch

    ref = torch.tensor([[[1.0, -2.0]], [[1e-3, 0.0]]], dtype=torch.float64)
    got = ref.clone()
    got[0, 0, 1] += 2e-6   # 1e-6 of problem 0's scale
    got[1, 0, 0] += 1e-7   # 1e-4 of problem 1's scale, 5e-8 of the batch's
    assert abs(bench.worst_rel_grad_err(got, ref) - 1e-4) < 1e-12
