"""GPU parity of the batched path (many independent Gaussian problems in one
pass) against the FP64 oracle, problem by problem. Sizes are ragged and not
multiples of the 256-point padding block, so every problem has padding
points; the ranges differ per problem.

Bars: FP64 NLL relative 1e-10 and gradient 1e-8 of max|g| (as for one
problem); FP32 NLL 1e-5 of the magnitude of
the NLL's terms (see test_gpu_factor.py) and gradient 1e-3 of max|g|."""
import numpy as np
import pytest
import torch

import vif_inputs as vi
from oracle import vif_oracle as vo
from tests.gpu_util import nbr_to_dev, nll_sum_magnitude, to_dev

pytestmark = pytest.mark.gpu

SIZES = [300, 1000, 257, 2000, 513, 256, 777]


def _problems(sizes, m=20, mv=8, seed=0):
    g = np.random.default_rng(seed)
    out = []
    for p, n in enumerate(sizes):
        rho = float(g.uniform(0.05, 0.2))
        w = vi.Workload(f"batch {p}", 4, n, 2, m, mv, vo.MATERN32, 1.0, np.array([rho]), 0.05, 0.0, "gaussian",
                        "subset")
        X = vi.coords(w, 100 + p)
        Z = vi.inducing_points(w, X, 100 + p)
        model = vo.Model(w.kernel, 1.0, w.lengthscales, 0.05)
        nbr = vo.neighbours(model, X, vo.inducing(model, X, Z), mv)
        L = np.linalg.cholesky(vo.cov(model, X, X) + 0.05 * np.eye(n))
        y = L @ vi.normals(w, n, problem=100 + p)
        theta = np.array([1.3, 0.8 * rho, 1.5 * 0.05])  # perturbed: gradient far from 0
        out.append((w, X, Z, nbr, y, theta))
    return out


def _batch_inputs(probs):
    X = np.concatenate([p[1] for p in probs])
    Z = np.concatenate([p[2] for p in probs])
    nbr = np.concatenate([p[3] for p in probs]).astype(np.int32)
    y = np.concatenate([p[4] for p in probs])
    theta = np.stack([p[5] for p in probs])
    return to_dev(X), to_dev(Z), nbr_to_dev(nbr), theta, to_dev(y)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_oracle(prec):
    from paper_2507_05064_amd.vif import VifBatch
    probs = _problems(SIZES)
    print(f"[gpu] batch {len(SIZES)} problems {prec}", flush=True)
    bt = VifBatch(SIZES, 2, 20, 8, precision=prec)
    Xd, Zd, nd, theta, yd = _batch_inputs(probs)
    nll, g = bt.nll_grad(Xd, Zd, nd, theta, yd)
    for k, (w, X, Z, nbr, y, th) in enumerate(probs):
        model = vo.Model.from_theta(w.kernel, th)
        nll_o, g_o = vo.nll_gaussian_grad(model, X, Z, nbr, y)
        if prec == "fp64":
            assert abs(nll[k] - nll_o) <= 1e-10 * abs(nll_o), (k, nll[k], nll_o)
            assert np.max(np.abs(g[k] - g_o)) <= 1e-8 * np.max(np.abs(g_o)), (k, g[k], g_o)
        else:
            S = nll_sum_magnitude(model, X, Z, nbr, y)
            assert abs(nll[k] - nll_o) <= 1e-5 * S, (k, nll[k], nll_o, S)
            assert np.max(np.abs(g[k] - g_o)) <= 1e-3 * np.max(np.abs(g_o)), (k, g[k], g_o)
    # NLL alone, and a repeated call, give the same numbers (fixed-order sums)
    nll2, none = bt.nll_grad(Xd, Zd, nd, theta, yd, grad=False)
    assert none is None and np.array_equal(nll2, nll)
    nll3, g3 = bt.nll_grad(Xd, Zd, nd, theta, yd)
    assert np.array_equal(nll3, nll) and np.array_equal(g3, g)


def test_batch_single_problem_equals_context():
    """A batch of one problem agrees with the single-problem context (FP64)."""
    from paper_2507_05064_amd.vif import VifBatch, VifContext
    probs = _problems([1234], seed=3)
    w, X, Z, nbr, y, th = probs[0]
    bt = VifBatch([w.n], 2, 20, 8, precision="fp64")
    nll_b, g_b = bt.nll_grad(*_batch_inputs(probs))
    ctx = VifContext(w.n, 2, 20, 8, kernel=w.kernel, precision="fp64")
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), th)
    nll_c, g_c = ctx.nll_grad(to_dev(y), 3)
    assert abs(nll_b[0] - nll_c) <= 1e-12 * abs(nll_c)
    assert np.max(np.abs(g_b[0] - g_c)) <= 1e-10 * np.max(np.abs(g_c))


def test_batch_rejects_bad_neighbour():
    from paper_2507_05064_amd.vif import VifBatch, VifError
    probs = _problems([300, 400], seed=5)
    probs[1][3][50, 0] = 50  # not an earlier point of its problem
    bt = VifBatch([300, 400], 2, 20, 8, precision="fp64")
    with pytest.raises(VifError) as e:
        bt.nll_grad(*_batch_inputs(probs))
    assert e.value.code == 1
