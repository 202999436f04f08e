"""GPU tests of the mixed-precision sweeps against the FP64 oracle.

prec = MACH_BF16: the sparse TTM's factor entries rounded to bfloat16 and
the sweep Gram's inputs rounded to bfloat16 (MFMA, float32 accumulation);
prec = MACH_FP8E4M3: the same factor entries, and the Gram's inputs in OCP
e4m3 with one scale (amax / 448) per staged tile.  The eigensolve stays in
float64 either way.

The stated bound: rounding with unit roundoff u perturbs the Gram of Y_(n)
by at most about 2 u ||Y_(n)||_F^2, so by Davis-Kahan a sweep's subspace
moves by at most 4 u ||Y_(n)||_F^2 / (lambda_r - lambda_{r+1}) (u = 2^-8
for bfloat16, products of two rounded values; u = 2^-4 for e4m3, three
mantissa bits).  Each sweep is checked within max(1e-3, that bound); after a
free run (HOSVD + 3 sweeps) the reconstruction error must be at most 1.01
times the oracle's (equal stated accuracy)."""
import numpy as np
import pytest

from oracle import mach as O
from tests.gpu_helpers import load_factors, project, recon_rel_error, say, sin_theta
from tests.test_gpu_solver import _setup

pytestmark = pytest.mark.gpu

UNIT = {"bf16": 2.0 ** -8, "fp8": 2.0 ** -4}


def _tol(Yn, r, u):
    return max(1e-3, min(1.0, 4.0 * O.davis_kahan_bound(Yn, r, u)))


def _prec(M, name):
    return {"bf16": M.MACH_BF16, "fp8": M.MACH_FP8E4M3}[name]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("name", ["tucker-64x32x48-f64", "monitor-32x16x2048", "voxel-16x16x16x64",
                                  "rowside96-96x12x12"])
def test_mixed_sweeps_within_stated_bound(name, prec):
    """Each mixed sweep starts from the oracle's factors and is compared with
    the oracle's FP64 sweep from the same factors; then a free-running run
    (HOSVD + 3 sweeps) against the oracle's run by reconstruction error."""
    from paper_0909_4969_amd import mach as M
    X, Xh, ranks, p, dec = _setup(name)
    code, u = _prec(M, prec), UNIT[prec]
    dec.hosvd()
    A_ref = O.hosvd_factors(Xh, ranks)
    worst = 0.0
    for it in range(3):
        load_factors(dec, A_ref)
        say(prec, "sweep", name, it)
        dec.sweep(prec=code)
        assert dec.status()[0] == 0
        A = [np.array(a) for a in A_ref]
        for n in range(len(ranks)):
            Yn = O.unfold(O.ttm_chain(Xh, A, n), n)
            A[n] = O.leading_left_singular_vectors(Yn, ranks[n])[0]
            A_g = dec.factors[n].cpu().numpy()
            np.testing.assert_allclose(A_g.T @ A_g, np.eye(ranks[n]), atol=1e-12)
            s, tol = sin_theta(A[n], A_g), _tol(Yn, ranks[n], u)
            worst = max(worst, s)
            say(f"  sweep {it} mode {n}: sin_theta {s:.3e} bound {tol:.2e}")
            assert s <= tol, (it, n, s, tol)
        A_ref, _ = O.hooi_sweep(Xh, A_ref, ranks)
    say(prec, "free run", name)
    dec.hosvd()
    for _ in range(3):
        dec.sweep(prec=code)
    assert dec.status()[0] == 0
    A_g = [a.cpu().numpy() for a in dec.factors]
    e_o = O.rel_error(X, O.core(Xh, A_ref), A_ref)
    e_g = recon_rel_error(X, project(Xh, A_g), A_g)
    say(f"  rel error {prec} {e_g:.6f} oracle {e_o:.6f}; worst sweep sin_theta {worst:.2e}")
    assert e_g <= 1.01 * e_o + 1e-6, (e_g, e_o)


def test_unsupported_precision_is_rejected():
    from paper_0909_4969_amd import mach as M
    X, Xh, ranks, p, dec = _setup("tucker-64x32x48-f64")
    dec.hosvd()
    with pytest.raises(M.MachError) as e:
        dec.sweep(prec=M.MACH_F64)
    assert e.value.code == M.MACH_EUNSUPPORTED
