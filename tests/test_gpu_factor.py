"""GPU parity of the factor build, neighbour selection and Gaussian NLL
against the FP64 oracle (same seeded inputs on both sides).

Tolerances (FP64 form): neighbour sets identical except near-ties within
the keys' rounding bound; A_i within 1e-10 of max|A| and D_i within 1e-10
relative; NLL within 1e-10 relative. FP32 form: NLL within 1e-5 of S, the
sum of the magnitudes of the terms the NLL adds up (nll_sum_magnitude):
the proposed FP32 bar of 1e-5 relative, taken relative to the sum's own
scale, which is |NLL| when the terms do not cancel and far more than |NLL|
when they do (the n = 1500 case below has NLL = -14 from terms of total
magnitude ~1.6e3); gradient within 1e-3 of max|g|. The plain relative bar
|NLL_fp32 - NLL| <= 1e-5 |NLL| is checked at the n = 100k workload's true
parameters (test_gpu_c2_true_theta.py).
BF16-input form: V is rounded to BF16 (unit roundoff 2^-9 = 2e-3) before
the per-point Gram, so an entry of the residual covariance K - V V^T moves
by up to ~2^-9 |V_a| |V_b| against conditional variances of the order of
the nugget (0.01-0.05). The form is checked against the oracle evaluated
with the same BF16 rounding of V (nll_gaussian_rounded_v with bf16_round),
where only the FP32 arithmetic differs: the FP32 bar, 1e-5 of S. Its
distance from the unrounded oracle is the rounding's, not the kernels': it
is printed and held to 5e-3 of S (NLL) and 5e-2 of max|g|; the 1e-3
relative proposed for the form's NLL is missed at some workloads (2.4e-3
at the n = 100k workload's true parameters).
"""
import numpy as np
import pytest
import torch

import vif_inputs as vi
from oracle import vif_oracle as vo
from tests import dense_ref as dr
from tests.gpu_util import compare_neighbour_sets, factor_rel_err, nbr_to_dev, nll_sum_magnitude, problem, to_dev

pytestmark = pytest.mark.gpu


def _ctx(w, n=None, m=None, mv=None, precision="fp64"):
    from paper_2507_05064_amd.vif import VifContext
    return VifContext(n or w.n, w.d, w.m if m is None else m, w.m_v if mv is None else mv, kernel=w.kernel,
                      likelihood=w.likelihood, precision=precision, tau_m=w.tau_m)


def _y_exact(model, X, seed):
    C = dr.exact_cov(model, X)
    return np.linalg.cholesky(C) @ np.random.default_rng(seed).standard_normal(X.shape[0])


@pytest.fixture(scope="module")
def c1():
    w = vi.config1()
    X, Z, model = problem(w)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, w.m_v)
    y = _y_exact(model, X, 11)
    return w, X, Z, model, ind, nbr, y


def test_c1_neighbours(c1):
    w, X, Z, model, ind, nbr_o, y = c1
    print(f"[gpu] C1 neighbours n={w.n} m={w.m} m_v={w.m_v}", flush=True)
    ctx = _ctx(w)
    nbr_g = ctx.select_neighbors(to_dev(X), to_dev(Z), w.theta).cpu().numpy()
    exact, ties = compare_neighbour_sets(model, X, ind, nbr_o, nbr_g)
    assert exact + ties == w.n
    assert ties <= 2


def test_c1_factor_and_nll_fp64(c1):
    w, X, Z, model, ind, nbr, y = c1
    print(f"[gpu] C1 factor/NLL fp64", flush=True)
    fac = vo.vecchia_factor(model, X, ind, nbr)
    nll_o = vo.nll_gaussian(model, X, Z, nbr, y).nll
    ctx = _ctx(w)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    A_g, D_g = (t.cpu().numpy() for t in ctx.export_factor())
    ea, ed = factor_rel_err(A_g, D_g, fac.A, fac.D)
    assert ea <= 1e-10 and ed <= 1e-10, (ea, ed)
    nll_g = ctx.nll(to_dev(y))
    assert abs(nll_g - nll_o) <= 1e-10 * abs(nll_o), (nll_g, nll_o)


def test_c1_nll_fp32(c1):
    w, X, Z, model, ind, nbr, y = c1
    print(f"[gpu] C1 NLL fp32", flush=True)
    nll_o = vo.nll_gaussian(model, X, Z, nbr, y).nll
    ctx = _ctx(w, precision="fp32")
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    nll_g = ctx.nll(to_dev(y))
    S = nll_sum_magnitude(model, X, Z, nbr, y)
    print(f"[gpu]   fp32 NLL err {abs(nll_g - nll_o) / S:.3e} of S ({abs(nll_g - nll_o) / abs(nll_o):.3e} relative)",
          flush=True)
    assert abs(nll_g - nll_o) <= 1e-5 * S, (nll_g, nll_o)


def test_c1_nll_bf16_input(c1):
    w, X, Z, model, ind, nbr, y = c1
    print(f"[gpu] C1 NLL bf16_in", flush=True)
    nll_o = vo.nll_gaussian(model, X, Z, nbr, y).nll
    nll_r = vo.nll_gaussian_rounded_v(model, X, Z, nbr, y, vo.bf16_round)
    ctx = _ctx(w, precision="bf16_in")
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    nll_g = ctx.nll(to_dev(y))
    S = nll_sum_magnitude(model, X, Z, nbr, y)
    print(f"[gpu]   bf16 NLL err vs rounded oracle {abs(nll_g - nll_r) / S:.3e} of S, "
          f"vs unrounded {abs(nll_g - nll_o) / S:.3e} of S ({abs(nll_g - nll_o) / abs(nll_o):.3e} relative)", flush=True)
    assert abs(nll_g - nll_r) <= 1e-5 * S, (nll_g, nll_r)
    assert abs(nll_g - nll_o) <= 5e-3 * S, (nll_g, nll_o)
    # the FP32 form on the same inputs is closer to the oracle: the BF16
    # rounding of V is what moves the result
    ctx32 = _ctx(w, precision="fp32")
    ctx32.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    assert abs(ctx32.nll(to_dev(y)) - nll_o) < abs(nll_g - nll_o)


def test_bf16_input_form_rejects_other_entry_points(c1):
    from paper_2507_05064_amd.vif import VifError
    w, X, Z, model, ind, nbr, y = c1
    ctx = _ctx(w, precision="bf16_in")
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    with pytest.raises(VifError) as e:
        ctx.laplace_mode(to_dev(y))
    assert e.value.code == 1 and "BF16-input" in str(e.value)


@pytest.mark.parametrize("n,m,mv", [(1, 0, 5), (2, 1, 3), (7, 3, 10), (33, 5, 15), (300, 0, 12),
                                    (300, 17, 0), (517, 33, 31), (2500, 200, 20)])
def test_shapes_and_edges_fp64(n, m, mv):
    """Ragged heads, n < m_v, no inducing points (classical Vecchia), no
    neighbours (FITC), m not a multiple of 16, 31 neighbours (two MFMA row
    blocks), several point tiles."""
    w = vi.scaled(vi.config2(), n, m=m, m_v=mv)
    print(f"[gpu] shapes n={n} m={m} m_v={mv}", flush=True)
    X, Z, model = problem(w)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    y = np.random.default_rng(n).standard_normal(n)
    ctx = _ctx(w)
    Xd, Zd = to_dev(X), to_dev(Z) if m else None
    if mv:
        nbr_g = ctx.select_neighbors(Xd, Zd, w.theta).cpu().numpy()
        exact, ties = compare_neighbour_sets(model, X, ind, nbr, nbr_g)
        assert exact + ties == n
    ctx.build_factor(Xd, Zd, nbr_to_dev(nbr) if mv else None, w.theta)
    A_g, D_g = (t.cpu().numpy() for t in ctx.export_factor())
    fac = vo.vecchia_factor(model, X, ind, nbr)
    ea, ed = factor_rel_err(A_g, D_g, fac.A, fac.D)
    assert ea <= 1e-10 and ed <= 1e-10, (ea, ed)
    nll_o = vo.nll_gaussian(model, X, Z, nbr, y).nll
    nll_g = ctx.nll(to_dev(y))
    assert abs(nll_g - nll_o) <= 1e-10 * abs(nll_o), (nll_g, nll_o)


def test_full_conditioning_equals_exact_gp_on_gpu():
    """m_v = n - 1 (n = 32): the GPU NLL equals the dense exact GP NLL."""
    n = 32
    w = vi.scaled(vi.config1(), n, m=6, m_v=n - 1)
    X, Z, model = problem(w)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, n - 1)
    y = _y_exact(model, X, 5)
    ctx = _ctx(w)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    ref = dr.gaussian_nll_dense(dr.exact_cov(model, X), y)
    assert abs(ctx.nll(to_dev(y)) - ref) <= 1e-10 * abs(ref)


def test_invalid_neighbour_list_is_rejected():
    from paper_2507_05064_amd.vif import VifError
    w = vi.scaled(vi.config1(), 50, m=5, m_v=4)
    X, Z, model = problem(w)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, 4)
    nbr[30, 1] = 30  # not an earlier point
    ctx = _ctx(w)
    with pytest.raises(VifError) as e:
        ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    assert e.value.code == 1 and "point 30" in str(e.value)


def test_not_pd_is_reported():
    from paper_2507_05064_amd.vif import VifError
    w = vi.scaled(vi.config1(), 60, m=0, m_v=5)
    X, Z, model = problem(w)
    X[40] = X[7]
    model0 = vo.Model(model.kernel, model.sigma1_sq, model.ls, 0.0)
    ind = vo.inducing(model0, X, Z)
    nbr = vo.neighbours(model0, X, ind, 5)
    ctx = _ctx(w)
    theta = w.theta.copy()
    theta[-1] = 0.0
    with pytest.raises(VifError) as e:
        ctx.build_factor(to_dev(X), None, nbr_to_dev(nbr), theta)
    assert e.value.code == 3 and "point 40" in str(e.value)


@pytest.mark.parametrize("n,m,mv,prec", [(400, 20, 8, "fp64"), (1500, 50, 10, "fp64"), (517, 33, 30, "fp64"),
                                              (300, 0, 6, "fp64"), (300, 17, 0, "fp64"), (1500, 50, 10, "fp32"),
                                         (1500, 50, 10, "bf16_in"), (517, 33, 30, "bf16_in")])
def test_gradient_matches_oracle(n, m, mv, prec):
    """Adjoint gradient (GPU) vs the oracle's forward-mode gradient at a
    perturbed theta (1.3 sigma1^2, 0.8 range, 1.5 nugget) where the gradient
    is far from zero. FP64: relative 1e-8 of max|g|; FP32: 1e-3 of max|g|;
    BF16-input: 5e-2 of max|g|."""
    w = vi.scaled(vi.config1(), n, m=m, m_v=mv)
    X, Z, model = problem(w)
    theta = w.theta * np.array([1.3, 0.8, 1.5])
    model = vo.Model.from_theta(w.kernel, theta, w.tau_m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    y = _y_exact(vo.Model.from_theta(w.kernel, w.theta), X, 21)
    print(f"[gpu] gradient n={n} m={m} m_v={mv} {prec}", flush=True)
    nll_o, g_o = vo.nll_gaussian_grad(model, X, Z, nbr, y)
    ctx = _ctx(w, precision=prec)
    ctx.build_factor(to_dev(X), to_dev(Z) if m else None, nbr_to_dev(nbr) if mv else None, theta)
    nll_g, g_g = ctx.nll_grad(to_dev(y), 3)
    tol = {"fp64": 1e-8, "fp32": 1e-3, "bf16_in": 5e-2}[prec]
    nerr = abs(nll_g - nll_o)
    S = nll_sum_magnitude(model, X, Z, nbr, y)
    print(f"[gpu]   NLL err {nerr / abs(nll_o):.3e} relative, {nerr / S:.3e} of S; "
          f"grad err {np.max(np.abs(g_g - g_o)) / np.max(np.abs(g_o)):.3e}", flush=True)
    if prec == "fp64":
        assert nerr <= 1e-10 * abs(nll_o), (nll_g, nll_o)
    elif prec == "fp32":
        assert nerr <= 1e-5 * S, (nll_g, nll_o, S)
    else:
        nll_r = vo.nll_gaussian_rounded_v(model, X, Z, nbr, y, vo.bf16_round)
        assert abs(nll_g - nll_r) <= 1e-5 * S, (nll_g, nll_r, S)
        assert nerr <= 5e-3 * S, (nll_g, nll_o, S)
    assert np.max(np.abs(g_g - g_o)) <= tol * np.max(np.abs(g_o)), (g_g, g_o)
    # a second call on the same factor is bit-identical (no atomics in the sums)
    nll_2, g_2 = ctx.nll_grad(to_dev(y), 3)
    assert nll_2 == nll_g and np.array_equal(g_2, g_g)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16_in"])
def test_repeated_gradient_evaluations_match_fresh_contexts(prec):
    """After its first gradient a context starts the derivative whitening of
    each later build on a second stream; a sequence of build + gradient (and
    a build followed by NLL only) on one context gives the same values as a
    fresh context per theta, bit for bit."""
    w = vi.scaled(vi.config1(), 1200, m=40, m_v=12)
    X, Z, model = problem(w)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, w.m_v)
    y = _y_exact(model, X, 5)
    thetas = [w.theta * np.array(f) for f in ([1.0, 1.0, 1.0], [1.3, 0.8, 1.5], [0.7, 1.2, 0.9], [1.1, 0.9, 1.2])]
    print(f"[gpu] repeated gradients n={w.n} m={w.m} m_v={w.m_v} {prec}", flush=True)
    shared = _ctx(w, precision=prec)
    dX, dZ, dN, dy = to_dev(X), to_dev(Z), nbr_to_dev(nbr), to_dev(y)
    for k, th in enumerate(thetas):
        shared.build_factor(dX, dZ, dN, th)
        if k == 2:  # NLL only: the started whitening is waited for by the next build
            shared.nll(dy)
            continue
        got = shared.nll_grad(dy, 3)
        fresh = _ctx(w, precision=prec)
        fresh.build_factor(dX, dZ, dN, th)
        ref = fresh.nll_grad(dy, 3)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1]), (k, got, ref)


def test_gradient_rejects_31_neighbours():
    """The adjoint joins one extra row to the 32-row per-point Gram: m_v <= 30."""
    from paper_2507_05064_amd.vif import VifError
    w = vi.scaled(vi.config1(), 100, m=8, m_v=31)
    X, Z, model = problem(w)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, 31)
    ctx = _ctx(w)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    with pytest.raises(VifError) as e:
        ctx.nll_grad(to_dev(np.zeros(100)), 3)
    assert e.value.code == 1


def test_autograd_function_matches_oracle_and_finite_differences():
    """torch.autograd through VifNLLFunction: the gradient equals the oracle's
    forward-mode gradient, and central differences of the GPU NLL agree with
    it (step 1e-5 relative, FP64)."""
    import torch
    from paper_2507_05064_amd.vif import vif_nll
    w = vi.scaled(vi.config1(), 400, m=20, m_v=10)
    X, Z, model = problem(w)
    theta0 = w.theta * np.array([1.3, 0.8, 1.5])
    model = vo.Model.from_theta(w.kernel, theta0, w.tau_m)
    nbr = vo.neighbours(model, X, vo.inducing(model, X, Z), 10)
    y = _y_exact(vo.Model.from_theta(w.kernel, w.theta), X, 5)
    _, g_o = vo.nll_gaussian_grad(model, X, Z, nbr, y)
    ctx = _ctx(w)
    Xd, Zd, nd, yd = to_dev(X), to_dev(Z), nbr_to_dev(nbr), to_dev(y)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    out = vif_nll(theta, ctx, Xd, Zd, nd, yd)
    (2.0 * out).backward()
    g = theta.grad.numpy() / 2.0
    assert np.max(np.abs(g - g_o)) <= 1e-8 * np.max(np.abs(g_o)), (g, g_o)
    for k in range(3):
        h = 1e-5 * theta0[k]
        tp, tm = theta0.copy(), theta0.copy()
        tp[k] += h
        tm[k] -= h
        fp = vif_nll(torch.tensor(tp), ctx, Xd, Zd, nd, yd).item()
        fm = vif_nll(torch.tensor(tm), ctx, Xd, Zd, nd, yd).item()
        assert abs((fp - fm) / (2 * h) - g[k]) <= 1e-5 * max(abs(g[k]), 1.0), (k, (fp - fm) / (2 * h), g[k])
