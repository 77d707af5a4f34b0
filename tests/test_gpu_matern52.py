"""GPU parity with the Matern-5/2 kernel (r(t) = (1 + sqrt5 t + 5 t^2 / 3)
e^{-sqrt5 t}): correlation neighbours as sets against the oracle's brute
force (near-ties within the keys' rounding bound accepted), the Gaussian NLL and adjoint
gradient at a perturbed theta against the oracle's forward-mode gradient
(FP64: 1e-10 relative NLL and 1e-8 of max|g|; FP32 form: 1e-5 of the
magnitude of the NLL's terms, see test_gpu_factor.py, and 1e-3),
and the Bernoulli-logit Laplace mode against the oracle's (1e-8)."""
import dataclasses

import numpy as np
import pytest

import vif_inputs as vi
from oracle import vif_oracle as vo
from tests import dense_ref as dr
from tests.gpu_util import compare_neighbour_sets, nbr_to_dev, nll_sum_magnitude, problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,mv,prec", [(1200, 30, 12, "fp64"), (1200, 30, 12, "fp32"), (400, 0, 8, "fp64")])
def test_matern52_neighbours_nll_grad(n, m, mv, prec):
    from paper_2507_05064_amd.vif import VifContext
    w = dataclasses.replace(vi.scaled(vi.config1(), n, m=m, m_v=mv), kernel=vo.MATERN52)
    X, Z, _ = problem(w)
    theta = w.theta * np.array([1.3, 0.8, 1.5])
    model = vo.Model.from_theta(w.kernel, theta, w.tau_m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    C = dr.exact_cov(vo.Model.from_theta(w.kernel, w.theta), X)
    y = np.linalg.cholesky(C) @ np.random.default_rng(n + m).standard_normal(n)
    nll_o, g_o = vo.nll_gaussian_grad(model, X, Z, nbr, y)
    print(f"[gpu] matern52 n={n} m={m} m_v={mv} {prec}", flush=True)
    ctx = VifContext(n, w.d, m, mv, kernel="matern52", precision=prec)
    nbr_g = ctx.select_neighbors(to_dev(X), to_dev(Z) if m else None, theta).cpu().numpy()
    exact, ties = compare_neighbour_sets(model, X, ind, nbr, nbr_g)
    assert exact + ties == n
    ctx.build_factor(to_dev(X), to_dev(Z) if m else None, nbr_to_dev(nbr), theta)
    nll_g, g_g = ctx.nll_grad(to_dev(y), 3)
    if prec == "fp64":
        assert abs(nll_g - nll_o) <= 1e-10 * abs(nll_o), (nll_g, nll_o)
        assert np.max(np.abs(g_g - g_o)) <= 1e-8 * np.max(np.abs(g_o)), (g_g, g_o)
    else:
        S = nll_sum_magnitude(model, X, Z, nbr, y)
        print(f"[gpu]   fp32 NLL err {abs(nll_g - nll_o) / S:.3e} of S", flush=True)
        assert abs(nll_g - nll_o) <= 1e-5 * S, (nll_g, nll_o, S)
        assert np.max(np.abs(g_g - g_o)) <= 1e-3 * np.max(np.abs(g_o)), (g_g, g_o)


def test_matern52_laplace_mode():
    from oracle import laplace_oracle as lo
    from tests.test_gpu_laplace import _ctx, _problem
    w, X, Z, model, nbr, prior, y = _problem(lo.BERNOULLI_LOGIT, 800, 20, 10, kernel=vo.MATERN52, ls=(0.1,))
    ref = lo.find_mode(prior, lo.BERNOULLI_LOGIT, y, tol=1e-14, solver="dense")
    print("[gpu] matern52 laplace mode n=800", flush=True)
    ctx = _ctx(w, lo.BERNOULLI_LOGIT, cg_tol=1e-12, cg_maxit=5000, newton_tol=1e-14)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    mode, st, _ = ctx.laplace_mode(to_dev(y))
    mode = mode.cpu().numpy()
    err = np.max(np.abs(mode - ref.mode)) / np.max(np.abs(ref.mode))
    print(f"[gpu] err {err:.3e} psi gpu {st['psi']:.12e} oracle {ref.psi:.12e} newton {st['newton_iters']} "
          f"pcg {st['pcg_iters']} halvings {st['halvings']}", flush=True)
    assert err <= 1e-8, (err, st)
    assert st["converged"] and abs(st["psi"] - ref.psi) <= 1e-9 * abs(ref.psi)
