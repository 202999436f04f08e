"""GPU tests of the serving loop: a window's result is the same alone and in a
mix of concurrent windows (bit for bit: every window has its own
workspaces and the kernels are deterministic); warm-started windows follow
the oracle's own chain (a stream's first window: HOSVD + sweeps; later
windows: time-mode update from the previous host/metric factors, then
sweeps) within 1e-5 in subspace angle where the eigengap at the oracle's
result is at least 1e-3 of the largest eigenvalue, else within the
Davis-Kahan bound; the HBM budget limits what is in flight."""
import numpy as np
import pytest

import synth
from oracle import mach as O
from tests.gpu_helpers import oracle_sweep_with_gaps, project, say, sin_theta, subspace_tol

pytestmark = pytest.mark.gpu

RANKS = (4, 2, 4)
P = 0.3
COLD, WARM = 3, 2


def _requests():
    reqs = []
    hosts = {0: 16, 1: 24, 2: 16}
    Ts = [256, 320, 288, 352, 300, 260]
    rid = 0
    for w in range(2):
        for s in range(3):
            reqs.append(synth.ServingRequest(rid, 0.0005 * rid, s, w, hosts[s], Ts[rid], 7000 + s))
            rid += 1
    return reqs


def _windows(reqs):
    import torch
    from paper_0909_4969_amd.serve import Window
    out, host = [], {}
    for r in reqs:
        X = synth.serving_window(r, metrics=8, ranks=RANKS)
        host[r.req_id] = X
        out.append(Window(r.req_id, r.stream_id, r.window_id, r.arrival_s, torch.from_numpy(X).cuda(), r.seed))
    return out, host


def _engine(**kw):
    from paper_0909_4969_amd.serve import Engine, ServeConfig
    cfg = ServeConfig(ranks=RANKS, p=P, sweeps_cold=COLD, sweeps_warm=WARM, **kw)
    return Engine(cfg)


def test_alone_equals_mix():
    reqs = _requests()
    wins, _ = _windows(reqs)
    say("serve mix", len(wins))
    mix = _engine(max_active=6, hip_streams=3).run(wins, realtime=False)
    assert any(r.warm for r in mix) and any(not r.warm for r in mix)
    for s in range(3):
        say("serve alone stream", s)
        alone = _engine(max_active=1, hip_streams=1).run([w for w in wins if w.stream_id == s],
                                                         realtime=False)
        for a in alone:
            m = mix[a.req_id]
            assert m.req_id == a.req_id and m.warm == a.warm and m.nnz == a.nnz
            for fa, fm in zip(a.factors, m.factors):
                assert bool((fa == fm).all()), (a.req_id, "factor differs")
            assert bool((a.core == m.core).all()), (a.req_id, "core differs")
            assert a.fit == m.fit


def test_warm_chain_matches_oracle():
    reqs = _requests()
    wins, host = _windows(reqs)
    say("serve oracle chain")
    res = _engine(max_active=4, hip_streams=2).run(wins, realtime=False)
    prev = {}
    for r in sorted(reqs, key=lambda q: (q.stream_id, q.window_id)):
        g = res[r.req_id]
        Xh = O.sampled_tensor(host[r.req_id], P, r.seed, r.window_id)
        n2 = float(np.sum(Xh * Xh))
        if r.stream_id in prev:
            assert g.warm
            A = [prev[r.stream_id][0], prev[r.stream_id][1], np.zeros((r.T, RANKS[2]))]
            A, tr = O.hooi_sweep(Xh, A, RANKS, first_mode=2)
            sweeps = WARM
        else:
            assert not g.warm
            A = O.hosvd_factors(Xh, RANKS)
            sweeps = COLD
        for _ in range(sweeps):
            A, tr = O.hooi_sweep(Xh, A, RANKS)
        prev[r.stream_id] = A
        fit_o = O.fit_from_norms(n2, tr[-1])
        A_g = [f.cpu().numpy() for f in g.factors]
        _, gaps, dk = oracle_sweep_with_gaps(Xh, A, RANKS)
        for n in range(3):
            s, tol = sin_theta(A[n], A_g[n]), subspace_tol(gaps[n], dk[n])
            say(f"  window {r.req_id} mode {n}: sin_theta {s:.2e} gap {gaps[n]:.2e} tol {tol:.1e}")
            assert s <= tol, (r.req_id, n, s, tol)
        assert abs(g.fit - fit_o) < 1e-5, (g.fit, fit_o)
        G_p = project(Xh, A_g)      # the core of the returned factors, formed on the host
        np.testing.assert_allclose(g.core.cpu().numpy(), G_p, rtol=0, atol=1e-5 * np.abs(G_p).max())


def test_hbm_budget_limits_inflight():
    reqs = _requests()
    wins, _ = _windows(reqs)
    eng = _engine(max_active=6, hip_streams=3)
    fps = [eng.footprint(w.X.shape) for w in wins]
    eng.cfg.hbm_budget = max(fps) + min(fps) // 2      # room for one window at a time
    say("serve budget", eng.cfg.hbm_budget)
    res = eng.run(wins, realtime=False)
    spans = sorted((r.admit_s, r.done_s) for r in res)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0, "two windows were in flight under a one-window budget"
    eng.cfg.hbm_budget = min(fps) - 1
    from paper_0909_4969_amd import mach as M
    with pytest.raises(M.MachError):
        eng.run(wins[:1], realtime=False)


def test_sliding_windows_with_stream_coins_match_oracle():
    """Overlapping windows of one stream (hop 150 ticks, length 400) sampled
    with stream coins (reading R9): each window's warm-started result follows
    the oracle's chain on the same tick-keyed samples."""
    import torch
    from paper_0909_4969_amd.serve import Window
    rng = np.random.default_rng(21)
    core = rng.standard_normal(RANKS)
    A_h = np.linalg.qr(rng.standard_normal((16, RANKS[0])))[0]
    A_m = np.linalg.qr(rng.standard_normal((8, RANKS[1])))[0]
    A_t = np.linalg.qr(rng.standard_normal((700, RANKS[2])))[0]
    Xl = np.einsum("abc,ia,jb,tc->ijt", core, A_h, A_m, A_t)
    Xl = (Xl + 0.01 * np.linalg.norm(Xl) / np.sqrt(Xl.size) * rng.standard_normal(Xl.shape)).astype(np.float32)
    seed, T, base = 4242, 400, 10_000
    wins, host = [], {}
    for w, t0 in enumerate((0, 150, 300)):
        X = np.ascontiguousarray(Xl[..., t0:t0 + T])
        host[w] = (X, base + t0)
        wins.append(Window(w, 0, w, 0.0, torch.from_numpy(X).cuda(), seed, tick0=base + t0))
    say("serve stream coins")
    res = _engine(max_active=3, hip_streams=2).run(wins, realtime=False)
    A = None
    for w in range(3):
        X, t0 = host[w]
        Xh = O.sampled_tensor_ticks(X, P, seed, t0)
        if A is None:
            A = O.hosvd_factors(Xh, RANKS)
            sweeps = COLD
        else:
            A = [A[0], A[1], np.zeros((T, RANKS[2]))]
            A, tr = O.hooi_sweep(Xh, A, RANKS, first_mode=2)
            sweeps = WARM
        for _ in range(sweeps):
            A, tr = O.hooi_sweep(Xh, A, RANKS)
        g = res[w]
        assert g.warm == (w > 0)
        assert g.nnz == int(np.count_nonzero(Xh))
        _, gaps, dk = oracle_sweep_with_gaps(Xh, A, RANKS)
        for n in range(3):
            s, tol = sin_theta(A[n], g.factors[n].cpu().numpy()), subspace_tol(gaps[n], dk[n])
            say(f"  window {w} mode {n}: sin_theta {s:.2e} gap {gaps[n]:.2e} tol {tol:.1e}")
            assert s <= tol, (w, n, s, tol)
        assert abs(g.fit - O.fit_from_norms(float(np.sum(Xh * Xh)), tr[-1])) < 1e-5


C5_RANKS, C5_P, C5_COLD, C5_WARM = (8, 4, 16), 0.05, 6, 3


def _c5_requests():
    """Serving windows of the Poisson-stream workload's shape: stream 0 has
    128 hosts (its host mode takes the short-side block iteration), stream 1
    has 32 hosts and windows of T >= 8192 ticks; two windows each (HOSVD
    start, then a warm start), 16 metrics, rank (8,4,16), p = 0.05."""
    spec = [(0, 128, 2048), (1, 32, 8192), (0, 128, 2500), (1, 32, 9000)]
    win = {0: 0, 1: 0}
    reqs = []
    for rid, (s, hosts, T) in enumerate(spec):
        reqs.append(synth.ServingRequest(rid, 0.0, s, win[s], hosts, T, 9100 + s))
        win[s] += 1
    return reqs


@pytest.mark.parametrize("prec", ["f32", "bf16", "fp8"])
def test_serving_windows_of_the_stream_workload_match_oracle(prec):
    """Each served window against the oracle's own warm-started chain on the
    same coins: float32 within the gap-aware subspace bar and the fit within
    1e-5; bfloat16 / e4m3 at equal stated accuracy, e <= 1.01 e_oracle
    (e = ||X - G x_n A_n|| / ||X||)."""
    import torch
    from paper_0909_4969_amd import mach as M
    from paper_0909_4969_amd.serve import Engine, ServeConfig, Window
    from tests.gpu_helpers import recon_rel_error
    code = {"f32": M.MACH_F32, "bf16": M.MACH_BF16, "fp8": M.MACH_FP8E4M3}[prec]
    reqs = _c5_requests()
    host = {r.req_id: synth.serving_window(r, metrics=16, ranks=C5_RANKS) for r in reqs}
    wins = [Window(r.req_id, r.stream_id, r.window_id, r.arrival_s, torch.from_numpy(host[r.req_id]).cuda(),
                   r.seed) for r in reqs]
    cfg = ServeConfig(ranks=C5_RANKS, p=C5_P, sweeps_cold=C5_COLD, sweeps_warm=C5_WARM, prec=code,
                      max_active=4, hip_streams=2)
    say("serve stream workload", prec, [tuple(w.X.shape) for w in wins])
    res = Engine(cfg).run(wins, realtime=False)
    prev = {}
    for r in sorted(reqs, key=lambda q: (q.stream_id, q.window_id)):
        g = res[r.req_id]
        X = host[r.req_id]
        Xh = O.sampled_tensor(X, C5_P, r.seed, r.window_id)
        n2 = float(np.sum(Xh * Xh))
        if r.stream_id in prev:
            assert g.warm
            A = [prev[r.stream_id][0], prev[r.stream_id][1], np.zeros((r.T, C5_RANKS[2]))]
            A, tr = O.hooi_sweep(Xh, A, C5_RANKS, first_mode=2)
            sweeps = C5_WARM
        else:
            assert not g.warm
            A = O.hosvd_factors(Xh, C5_RANKS)
            sweeps = C5_COLD
        for _ in range(sweeps):
            A, tr = O.hooi_sweep(Xh, A, C5_RANKS)
        prev[r.stream_id] = A
        A_g = [f.cpu().numpy() for f in g.factors]
        e_o = O.rel_error(X, O.core(Xh, A), A)
        e_g = recon_rel_error(X, g.core.cpu().numpy(), A_g)
        say(f"  window {r.req_id} ({X.shape}, {'warm' if g.warm else 'cold'}): e {e_g:.6f} oracle {e_o:.6f}")
        if prec == "f32":
            _, gaps, dk = oracle_sweep_with_gaps(Xh, A, C5_RANKS)
            for n in range(3):
                s, tol = sin_theta(A[n], A_g[n]), subspace_tol(gaps[n], dk[n])
                say(f"    mode {n}: sin_theta {s:.2e} gap {gaps[n]:.2e} tol {tol:.1e}")
                assert s <= tol, (r.req_id, n, s, tol)
            assert abs(g.fit - O.fit_from_norms(n2, tr[-1])) < 1e-5
        else:
            assert e_g <= 1.01 * e_o + 1e-7, (r.req_id, e_g, e_o)
