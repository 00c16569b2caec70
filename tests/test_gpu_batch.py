"""Batched HOPM (hopm_batch_prepare / hopm_batch_run through the C ABI):
every instance must match its own float64 oracle trajectory and a standalone
hopm_iterate run, deterministically, also when replayed from a hipGraph."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import hopm as H
from oracle import tvc as O
from paper_2501_03121_amd import batch as B
from paper_2501_03121_amd import synth
from _util import host

pytestmark = pytest.mark.gpu


def make_batch(dev, count, seed, hi=40, lo=3):
    rng = synth.rng(seed)
    As, x0s, exact = [], [], []
    for i in range(count):
        d = int(rng.integers(3, 6))
        dims = tuple(int(rng.integers(lo, hi + 1)) for _ in range(d))
        Ah = synth.normal(dims, seed * 1000 + i).astype(np.float32)
        As.append(torch.from_numpy(Ah).to(dev))
        exact.append(Ah.astype(np.float64))
        x0s.append(synth.unit_vectors(dims, seed * 1000 + 500 + i))
    return As, x0s, exact


@pytest.mark.parametrize("tile_elems", [64, 4096, 1 << 16])
def test_batch_matches_oracle(dev, tile_elems):
    As, x0s, exact = make_batch(dev, 24, 1, hi=20)
    xs = [tvc.pack_vectors(x0, dev) for x0 in x0s]
    sweeps = 4
    bp = B.prepare(As, xs, sweeps, tile_elems=tile_elems, grid=64)
    B.run(bp)
    torch.cuda.synchronize()
    assert B.error_word(bp) == 0
    res = B.results(bp)
    for i, (A, x0) in enumerate(zip(exact, x0s)):
        ref = H.hopm(A, x0, sweeps=sweeps)
        got = np.split(host(xs[i]), np.cumsum(A.shape)[:-1])
        for g, r in zip(got, ref.xs):
            assert np.linalg.norm(g - r) < 2e-5, (i, A.shape)
        assert abs(res[i].lam - ref.lam) < 2e-5 * ref.lam
        assert res[i].sweeps == sweeps and res[i].status == 0
        assert abs(res[i].delta - ref.deltas[-1]) < 2e-5 + 1e-3 * ref.deltas[-1]


def test_batch_equals_standalone_and_is_deterministic(dev):
    As, x0s, _ = make_batch(dev, 16, 2, hi=48)
    sweeps = 5
    xs = [tvc.pack_vectors(x0, dev) for x0 in x0s]
    bp = B.prepare(As, xs, sweeps, tile_elems=2048)
    B.run(bp)
    first = [x.clone() for x in xs]
    for x, x0 in zip(xs, x0s):
        x.copy_(tvc.pack_vectors(x0, dev))
    B.run(bp)
    torch.cuda.synchronize()
    assert B.error_word(bp) == 0
    for a, b in zip(first, xs):
        assert torch.equal(a, b)
    for A, x0, xb in zip(As, x0s, first):
        xi = tvc.pack_vectors(x0, dev)
        tvc.hopm_iterate(A, xi, sweeps)
        assert torch.allclose(xi, xb, atol=2e-5, rtol=0)


def test_batch_graph_replays(dev):
    As, x0s, exact = make_batch(dev, 20, 3, hi=32)
    sweeps = 3
    init = [tvc.pack_vectors(x0, dev) for x0 in x0s]
    xs = [v.clone() for v in init]
    bp = B.prepare(As, xs, sweeps, tile_elems=4096)

    def reset():
        for x, v in zip(xs, init):
            x.copy_(v)

    B.run(bp)
    torch.cuda.synchronize()
    eager = [x.clone() for x in xs]
    g = B.capture(bp, reset)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert B.error_word(bp) == 0
        for a, b in zip(eager, xs):
            assert torch.equal(a, b)
        # eager work between replays
        reset()
        B.run(bp)
        torch.cuda.synchronize()
        for a, b in zip(eager, xs):
            assert torch.equal(a, b)


def test_batch_planted_recovery(dev):
    # the batch workload's shape recipe, scaled down: orders 3..5, planted
    # rank-1 signal lambda ~ U[2, 20] on N(0,1) noise, warm start
    specs = synth.batch_instances(12, 7, lo=8, hi=64)
    As, xs, planted, lams = [], [], [], []
    for i, (dims, lam) in enumerate(specs):
        lam_big = lam * 20.0
        Ah, a = synth.planted_rank1(dims, lam_big, 1.0, 40 + i, noise_kind="normal", vec_kind="normal")
        As.append(torch.from_numpy(Ah.astype(np.float32)).to(dev))
        xs.append(tvc.pack_vectors(synth.warm_start(a, 0.9, 90 + i), dev))
        planted.append(a)
        lams.append(lam_big)
    bp = B.prepare(As, xs, 30, tile_elems=1024)
    B.run(bp)
    torch.cuda.synchronize()
    assert B.error_word(bp) == 0
    for i, r in enumerate(B.results(bp)):
        got = np.split(host(xs[i]), np.cumsum(specs[i][0])[:-1])
        assert min(abs(float(np.dot(g, v))) for g, v in zip(got, planted[i])) > 0.9
        assert abs(r.lam - lams[i]) < 0.2 * lams[i]


def test_batch_profile_counts_every_item(dev):
    # every queue slot is run exactly once: sweeps * (nt1 + nt2 + 2) per instance
    As, x0s, _ = make_batch(dev, 10, 4, hi=30)
    xs = [tvc.pack_vectors(x0, dev) for x0 in x0s]
    bp = B.prepare(As, xs, 3, tile_elems=512)
    B.run(bp)
    torch.cuda.synchronize()
    assert B.error_word(bp) == 0
    p = B.profile(bp)
    assert p["items"] == int(bp.plan.queue_slots)
    assert p["work_s"] > 0 and p["wait_s"] >= 0 and 0 < p["busy_fraction"] <= 1
