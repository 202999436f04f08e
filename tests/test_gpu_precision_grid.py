"""Precision grid on the full monitoring window (128 x 16 x 16384 float32,
rank (8,4,16)): keep probabilities p in {0.2, 0.05, 0.01} times sweep
precisions {float32, bfloat16, e4m3}, each HOSVD + 20 sweeps + core on the
device against the FP64 oracle's run on the same coins.

Reported per cell: the largest principal-angle sine per mode and the
reconstruction errors e = ||X - G x_n A_n|| / ||X|| of device and oracle.
Asserted: float32 reaches the oracle's e within 1e-5 (relative) and its fit
within 1e-5; the mixed precisions reach equal stated accuracy,
e <= 1.01 e_oracle."""
import numpy as np
import pytest

import synth
from oracle import mach as O
from tests.gpu_helpers import project, recon_rel_error, say, sin_theta

pytestmark = pytest.mark.gpu

SHAPE, RANKS, SWEEPS, SEED = (128, 16, 16384), (8, 4, 16), 20, 20264


@pytest.fixture(scope="module")
def window():
    X, _ = synth.workload2(SHAPE)
    return X


@pytest.mark.parametrize("p", [0.2, 0.05, 0.01])
def test_precision_grid(window, p):
    import torch
    from paper_0909_4969_amd import mach as M
    X = window
    Xh = O.sampled_tensor(X, p, SEED, 0)
    say(f"grid p {p}: oracle HOSVD + {SWEEPS} sweeps")
    n2 = float(np.sum(Xh * Xh))
    A_o = O.hosvd_factors(Xh, RANKS)
    for _ in range(SWEEPS):
        A_o, tr = O.hooi_sweep(Xh, A_o, RANKS)
    fit_o = O.fit_from_norms(n2, tr[-1])
    e_o = O.rel_error(X, O.core(Xh, A_o), A_o)
    del Xh
    dec = M.Decomposition(SHAPE, RANKS, p)
    Xd = torch.from_numpy(X).cuda()
    for name, code in (("f32", M.MACH_F32), ("bf16", M.MACH_BF16), ("fp8", M.MACH_FP8E4M3)):
        say(f"grid p {p} {name}: device HOSVD + {SWEEPS} sweeps + core")
        dec.sample(Xd, SEED, 0)
        dec.hosvd()
        for _ in range(SWEEPS):
            dec.sweep(prec=code)
        G = dec.core().cpu().numpy()
        assert dec.status()[0] == 0
        A_g = [a.cpu().numpy() for a in dec.factors]
        fit_g = float(dec.fit.item())
        e_g = recon_rel_error(X, G, A_g)
        sines = [sin_theta(a, b) for a, b in zip(A_o, A_g)]
        say(f"  p {p} {name}: sin_theta " + " ".join(f"{s:.2e}" for s in sines) +
            f"; e {e_g:.7f} oracle {e_o:.7f} ({(e_g - e_o) / e_o:+.2e}); fit {fit_g:.7f} oracle {fit_o:.7f}")
        if name == "f32":
            assert abs(e_g - e_o) <= 1e-5 * e_o, (e_g, e_o)
            assert abs(fit_g - fit_o) <= 1e-5, (fit_g, fit_o)
        else:
            assert e_g <= 1.01 * e_o, (name, e_g, e_o)
    del dec, Xd
    torch.cuda.synchronize()
