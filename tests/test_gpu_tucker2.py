"""GPU parity of Tucker2 (reading R11: the last mode left uncompressed,
identity factor, core R_1 x .. x R_{d-1} x I_d) against the FP64 oracle:
HOSVD factors of the compressed modes, one sweep from the oracle's factors,
the core from the same factors, and a free run (HOSVD + 3 sweeps) by fit and
reconstruction error.  Bars as for Tucker3: 1e-5 in subspace angle where
the relative eigengap is at least 1e-3 (else the Davis-Kahan bound), 1e-5
relative on the core, 1e-5 on fit and error."""
import numpy as np
import pytest

import synth
from oracle import mach as O
from tests.gpu_helpers import (columns_elementwise, load_factors, oracle_sweep_with_gaps, project,
                               recon_rel_error, rel, say, sin_theta, subspace_tol)

pytestmark = pytest.mark.gpu


def _sensor():
    X, _ = synth.workload1(shape=(54, 4, 600), ranks=(5, 2, 6), seed=81, rel_noise=0.05)
    return X.astype(np.float32), (5, 2, 0), 0.1, 91
def _monitor():
    X, _ = synth.workload2(shape=(32, 16, 2048), seed=82)
    return X, (8, 4, 0), 0.1, 92
def _monitor128():
    X, _ = synth.workload2(shape=(128, 16, 2048), seed=83)
    return X, (8, 4, 0), 0.1, 93
def _matrix():
    X, _ = synth.workload1(shape=(200, 300), ranks=(6, 6), seed=84, rel_noise=0.05)
    return X.astype(np.float32), (6, 0), 0.3, 94

# sensor-54x4x600: the paper's sensor layout (sensors x measurement types x
# ticks) with time uncompressed; monitor-128x16x2048: its host mode's Gram
# (side 128) takes the subspace iteration; matrix-200x300: d = 2.
CASES = {"sensor-54x4x600": _sensor, "monitor-32x16x2048": _monitor,
         "monitor-128x16x2048": _monitor128, "matrix-200x300": _matrix}


@pytest.mark.parametrize("name", list(CASES))
def test_tucker2_matches_oracle(name):
    import torch
    from paper_0909_4969_amd import mach as M
    X, ranks, p, seed = CASES[name]()
    d = len(ranks)
    dec = M.Decomposition(X.shape, ranks, p)
    Xd = torch.from_numpy(X).cuda()
    Xh = O.sampled_tensor(X, p, seed, 0)
    say("tucker2 hosvd", name, X.shape, ranks)
    dec.sample(Xd, seed, 0)
    dec.hosvd()
    assert dec.status()[0] == 0
    A_ref = O.hosvd_factors(Xh, ranks)
    assert A_ref[-1] is None
    for n in range(d - 1):
        A_g = dec.factors[n].cpu().numpy()
        Un = O.unfold(Xh, n)
        tol = subspace_tol(O.eigengap(Un, ranks[n]), O.davis_kahan_bound(Un, ranks[n], 2.0 ** -24))
        s = sin_theta(A_ref[n], A_g)
        say(f"  hosvd mode {n}: sin_theta {s:.3e} tol {tol:.1e}")
        np.testing.assert_allclose(A_g.T @ A_g, np.eye(ranks[n]), atol=1e-12)
        assert s <= tol, (n, s, tol)
    say("tucker2 one sweep", name)
    load_factors(dec, A_ref)
    dec.sweep()
    assert dec.status()[0] == 0
    sing = {}
    A_one, gaps, dk = oracle_sweep_with_gaps(Xh, A_ref, ranks, sing=sing)
    assert A_one[-1] is None
    for n in range(d - 1):
        A_g = dec.factors[n].cpu().numpy()
        s, tol = sin_theta(A_one[n], A_g), subspace_tol(gaps[n], dk[n])
        w = columns_elementwise(A_one[n], A_g, sing[n])
        say(f"  sweep mode {n}: sin_theta {s:.3e} gap {gaps[n]:.2e} tol {tol:.1e}; columns {w:.2e}")
        assert s <= tol, (n, s, tol)
        assert w <= 1.0, (n, w)
    say("tucker2 core", name)
    load_factors(dec, A_one)
    G = dec.core().cpu().numpy()
    assert dec.status()[0] == 0
    G_o = O.core(Xh, A_one)
    assert G.shape == G_o.shape == tuple(ranks[:-1]) + (X.shape[-1],)
    say(f"  core rel {rel(G, G_o):.2e}")
    assert rel(G, G_o) < 1e-5
    np.testing.assert_allclose(G, G_o, rtol=0, atol=1e-5 * np.abs(G_o).max())
    assert abs(float(dec.norm2.cpu()) - float(np.sum(G_o ** 2))) < 2e-5 * float(np.sum(G_o ** 2))
    say("tucker2 free run", name)
    dec.hosvd()
    for _ in range(3):
        dec.sweep()
    G_g = dec.core().cpu().numpy()
    assert dec.status()[0] == 0
    A_g = [f.cpu().numpy() if f.numel() else None for f in dec.factors]
    res = O.mach_hooi(X, ranks, p, seed, 0, sweeps=3, Xh=Xh)
    e_o = O.rel_error(X, res.core, res.factors)
    e_g = recon_rel_error(X, G_g, A_g)
    fit_g = float(dec.fit.cpu())
    say(f"  fit gpu {fit_g:.7f} oracle {res.fit_trace[-1]:.7f}; e gpu {e_g:.7f} oracle {e_o:.7f}")
    assert abs(fit_g - res.fit_trace[-1]) < 1e-5
    assert abs(e_g - e_o) <= 1e-5 * e_o
    assert rel(G_g, project(Xh, A_g)) < 1e-5
