"""GPU restarted GMRES (hh_solve) against the oracle's GMRES on the oracle's own
H_h matrix: same iteration count (within one step), solutions within a
tolerance set by the solver tolerance, and the true residual of the GPU's
solution, recomputed with the oracle's product, within the tolerance."""
import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O
from parity_util import build_pair, compare_structure, rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("trans", [False, True])
def test_gmres_gaussian_kernel_with_shift(trans):
    torch = _torch()
    rng = np.random.default_rng(3)
    P = rng.random((3000, 3))
    shift, rtol = 0.1, 1e-10
    g, o = build_pair(P, W.GAUSS, 1e-8, np.sqrt(3.0), -1, 64, h=0.1)
    compare_structure(g, o)
    b = rng.standard_normal(3000)
    x, it, rr = g.solve(torch.from_numpy(b).cuda(), shift=shift, rtol=rtol, restart=30,
                        max_iter=600, trans=trans)
    x = x.cpu().numpy()
    prod = (lambda v: O.matvec_t(o, v)) if trans else (lambda v: O.matvec(o, v))
    op = lambda v: prod(v) + shift * v
    xo, ito, hist = O.gmres(op, b, rtol=rtol, restart=30, max_iter=600)
    print(f"GMRES(30), trans={trans}: GPU {it} steps relres {rr:.2e}, oracle {ito} steps "
          f"relres {hist[-1]:.2e}, solutions differ by {rel(x, xo):.2e}", flush=True)
    assert abs(it - ito) <= 1
    assert rr <= rtol
    assert np.linalg.norm(b - op(x)) <= 2 * rtol * np.linalg.norm(b)
    assert rel(x, xo) <= 1e-7
    g.free()


def test_gmres_double_layer_transpose_and_initial_guess():
    torch = _torch()
    rng = np.random.default_rng(5)
    n = 2500
    P = np.concatenate([W.sphere_surface(n // 2, 3, rng), W.ball_interior(n - n // 2, 3, rng)])
    nrm = W.unit_normals(n, 3, rng)
    g, o = build_pair(P, W.DOUBLE_LAYER, 1e-8, 1.5, -1, 64, normals=nrm, mask=0x3)
    b = rng.standard_normal(n)
    # second-kind form: a shift of a few times ||H|| (nearby points make the
    # double-layer entries large), solved with the transpose, then refined from
    # the first solution as the initial guess
    shift = 1e6
    x1, it1, rr1 = g.solve(torch.from_numpy(b).cuda(), shift=shift, rtol=1e-6, restart=10, trans=True)
    x2, it2, rr2 = g.solve(torch.from_numpy(b).cuda(), x0=x1, shift=shift, rtol=1e-12, restart=10,
                           trans=True)
    assert rr1 <= 1e-6 and rr2 <= 1e-12 and it2 <= it1 + 10
    op = lambda v: O.matvec_t(o, v) + shift * v
    x = x2.cpu().numpy()
    assert np.linalg.norm(b - op(x)) <= 1e-11 * np.linalg.norm(b)
    g.free()
