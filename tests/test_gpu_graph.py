"""The HOOI sweeps of a window can be captured in a HIP graph (no memset
nodes, no host synchronisation, no allocation inside mach_hooi_sweep) and
replayed for later windows: every replay gives exactly the factors, fit and
core of the same sweeps launched one by one.  Replays alternate with eager
work and host synchronisation (sampling, HOSVD and the core of each window,
and the eager reference run)."""
import hashlib

import pytest

import synth
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

SHAPE, RANKS, P, SWEEPS, SEED = (32, 16, 2048), (8, 4, 16), 0.1, 5, 20262


def _digest(dec):
    h = hashlib.sha256()
    for a in dec.factors:
        h.update(a.cpu().numpy().tobytes())
    h.update(dec.fit.cpu().numpy().tobytes())
    h.update(dec.G.cpu().numpy().tobytes())
    return h.hexdigest()


def _window(dec, X, w, s, graph=None):
    import torch
    with torch.cuda.stream(s):
        dec.sample(X, SEED, w, stream=s)
        dec.hosvd(stream=s)
        if graph is not None:
            graph.replay()
        else:
            for _ in range(SWEEPS):
                dec.sweep(stream=s)
        dec.core(stream=s)
        st = dec.status(stream=s)[0]
    assert st == 0, st
    return _digest(dec)


def test_captured_sweeps_replay_exactly():
    import torch
    from paper_0909_4969_amd import mach as M
    X, _ = synth.workload2(shape=SHAPE, seed=5)
    X = torch.from_numpy(X).cuda()
    s = torch.cuda.Stream()
    dec = M.Decomposition(SHAPE, RANKS, P)
    _window(dec, X, 0, s)
    with torch.cuda.stream(s):
        dec.sample(X, SEED, 1, stream=s)
        dec.hosvd(stream=s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(SWEEPS):
            dec.sweep(stream=s)
    s.synchronize()
    for w in (2, 3, 4, 5):
        say(f"window {w}: eager sweeps, then the captured sweeps")
        eager = _window(dec, X, w, s)
        replay = _window(dec, X, w, s, graph=g)
        assert replay == eager, w
    del g
    torch.cuda.synchronize()
