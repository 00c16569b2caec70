"""Parity beyond order 6: the contraction in every mode and format for
orders 7-16 (the C ABI's limit), the paper's Table 1 hypersquare tensors
(orders 2-10, Sec. 5.1) at full size on sampled outputs, HOPM trajectories
at orders 7-10 and one full-size sweep of the 10^9 and 8^10 tensors, and
batched HOPM instances of orders 6-8, all against the float64 oracle.
Outputs are also checked one by one against the rounding bound of their
dot product."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import hopm as H
from oracle import tvc as O
from paper_2501_03121_amd import batch as B
from paper_2501_03121_amd import synth
from _util import TOL, assert_elementwise, host, stored_tensor, vec

pytestmark = pytest.mark.gpu

FMTS = ["f64", "f32", "f16", "bf16", "e4m3"]
# odd extents, so rows are rarely whole 16-byte vectors
HIGH_ORDER = [
    (3, 2, 5, 3, 2, 3, 7),
    (2, 3, 2, 5, 2, 3, 3, 5),
    (3, 2, 3, 2, 5, 2, 3, 2, 3),
    (2, 3, 2, 2, 3, 2, 2, 5, 2, 3),
    (2, 3, 2, 2, 3, 2, 2, 3, 2, 2, 3, 2),
    (2, 2, 3, 2, 2, 2, 2, 3, 2, 2, 2, 2, 2, 2, 2, 3),
]


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("dims", HIGH_ORDER, ids=lambda d: f"order{len(d)}")
def test_high_order_all_modes(dev, fmt, dims):
    A, S, exact = stored_tensor(dims, fmt, 17, dev)
    for k in range(len(dims)):
        x, xh = vec(dims[k], 70 + k, fmt, dev)
        y = tvc.contract(A, x, k, scale=S)
        ref = O.tvc(exact, xh, k)
        got = host(y)
        assert got.shape == ref.shape
        assert O.rel_err(got, ref) <= TOL[fmt], (fmt, dims, k)
        assert_elementwise(got, ref, O.tvc(np.abs(exact), np.abs(xh), k), dims[k], fmt, (dims, k))


TABLE1 = [(30623, 2), (979, 3), (175, 4), (63, 5), (31, 6), (19, 7), (13, 8), (10, 9), (8, 10)]
SAMPLES = 2048


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,d", TABLE1, ids=[f"{n}^{d}" for n, d in TABLE1])
def test_table1_full_size_sampled(dev, n, d):
    # float32 N(0,1) at the paper's Table 1 element counts, every mode, 2048
    # sampled outputs (plus the first and last) each computed by the oracle
    # from the exact host copy of the device bytes
    dims = (n,) * d
    A = synth.device_normal(dims, 40 + d, dev)
    Ah = A.cpu().numpy()
    for k in range(d):
        xh = synth.unit_vectors([n], 50 + k)[0].astype(np.float32)
        y = tvc.contract(A, torch.from_numpy(xh).to(dev), k)
        u, _, v = O.matricized_dims(dims, k)
        g = synth.rng(60 + k)
        lr = np.stack([g.integers(0, u, SAMPLES), g.integers(0, v, SAMPLES)], axis=1)
        lr = np.concatenate([lr, [[0, 0], [u - 1, v - 1]]])
        got = host(y).reshape(u, v)[lr[:, 0], lr[:, 1]]
        ref = O.tvc_sample(Ah, xh, k, lr)
        assert O.rel_err(got, ref) < 1e-5, (dims, k)
        ref_abs = O.tvc_sample(np.abs(Ah), np.abs(xh), k, lr)
        assert_elementwise(got, ref, ref_abs, n, "f32", (dims, k))
        del y
    del A
    torch.cuda.empty_cache()


# float64 at the paper's Table 1 element counts (6.6-8.6 GB), on the tensors
# whose float64 plans differ from float32's: column strips of four units per
# lane on odd row pitches (175^4, 63^5), the staged kernel with 64 KB blocks
# (10^9 modes 6-7) and with 4-unit slab rows (8^10 mode 8); sampled outputs of
# every mode as above, each within the float64 rounding bound of its dot product
F64_TABLE1 = [(175, 4), (63, 5), (10, 9), (8, 10)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,d", F64_TABLE1, ids=[f"{n}^{d}" for n, d in F64_TABLE1])
def test_table1_full_size_sampled_f64(dev, n, d):
    dims = (n,) * d
    A = synth.device_normal(dims, 40 + d, dev, dtype=torch.float64)
    Ah = A.cpu().numpy()
    Aabs = np.abs(Ah)
    for k in range(d):
        xh = synth.unit_vectors([n], 50 + k)[0]
        y = tvc.contract(A, torch.from_numpy(xh).to(dev), k)
        u, _, v = O.matricized_dims(dims, k)
        g = synth.rng(60 + k)
        lr = np.stack([g.integers(0, u, SAMPLES), g.integers(0, v, SAMPLES)], axis=1)
        lr = np.concatenate([lr, [[0, 0], [u - 1, v - 1]]])
        got = host(y).reshape(u, v)[lr[:, 0], lr[:, 1]]
        ref = O.tvc_sample(Ah, xh, k, lr)
        ref_abs = O.tvc_sample(Aabs, np.abs(xh), k, lr)
        assert_elementwise(got, ref, ref_abs, n, "f64", (dims, k))
        del y
    del A
    torch.cuda.empty_cache()


def run_sweeps(A, x0, sweeps, dev, scale=None):
    x = tvc.pack_vectors(x0, dev)
    out = []
    for _ in range(sweeps):
        r = tvc.read_stats(tvc.hopm_iterate(A, x, 1, scale=scale))
        out.append((host(x).copy(), r))
    return out


def check_against_oracle(traj, exact, x0, tol, form="chain"):
    dims = exact.shape
    xs = [np.asarray(v) for v in x0]
    for i, (xg, r) in enumerate(traj):
        o = H.hopm(exact, xs, sweeps=1, form=form, workers=16)
        xs = o.xs
        got = np.split(xg, np.cumsum(dims)[:-1])
        for j in range(len(dims)):
            assert np.linalg.norm(got[j] - xs[j]) <= tol, (i, j)
        assert abs(r.lam - o.lam) <= tol * o.lam, (i, r.lam, o.lam)
        assert r.status == 0


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("dims", HIGH_ORDER, ids=lambda d: f"order{len(d)}")
def test_hopm_high_order_trajectory(dev, fmt, dims):
    A, _, exact = stored_tensor(dims, fmt, 19, dev, kind="normal")
    x0 = synth.unit_vectors(dims, 20)
    check_against_oracle(run_sweeps(A, x0, 4, dev), exact, x0, 1e-11 if fmt == "f64" else 2e-5)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
def test_hopm_high_order_narrow_formats(dev, fmt):
    dims = (3, 4, 2, 3, 5, 2, 3, 4)
    A, S, exact = stored_tensor(dims, fmt, 21, dev, kind="normal")
    x0 = synth.unit_vectors(dims, 22)
    check_against_oracle(run_sweeps(A, x0, 3, dev, scale=S), exact, x0, 2e-5)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n,d", [(10, 9), (8, 10)], ids=["10^9", "8^10"])
def test_hopm_full_size_sweep_high_order(dev, n, d):
    # one sweep of the fused two-pass HOPM on 10^9 and 8^10 float32 tensors
    # against the oracle's canonical sweep (multilinear form, float64)
    dims = (n,) * d
    A = synth.device_normal(dims, 80 + d, dev)
    x0 = synth.unit_vectors(dims, 81 + d)
    traj = run_sweeps(A, x0, 1, dev)
    Ah = A.cpu().numpy()
    del A
    torch.cuda.empty_cache()
    check_against_oracle(traj, Ah, x0, 1e-5, form="kron")


def _batch(dev, count, seed, orders, lo, hi):
    rng = synth.rng(seed)
    As, x0s, exact = [], [], []
    for i in range(count):
        d = int(rng.choice(orders))
        dims = tuple(int(rng.integers(lo, hi + 1)) for _ in range(d))
        Ah = synth.normal(dims, seed * 1000 + i).astype(np.float32)
        As.append(torch.from_numpy(Ah).to(dev))
        exact.append(Ah.astype(np.float64))
        x0s.append(synth.unit_vectors(dims, seed * 1000 + 500 + i))
    return As, x0s, exact


@pytest.mark.parametrize("tile_elems", [256, 1 << 14])
def test_batch_orders_6_to_8(dev, tile_elems):
    As, x0s, exact = _batch(dev, 18, 5, (6, 7, 8), 2, 7)
    assert {a.dim() for a in As} == {6, 7, 8}
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


@pytest.mark.timeout(900)
def test_batch_recipe_slice_50_sweeps(dev):
    # instances of the 512-instance batch recipe (orders 3-5, every dim in
    # [16, floor(256^(3/d))], N(0,1) + lambda a o b o ..., lambda ~ U[2, 20]),
    # the four largest and four others, swept 50 times in one launch and
    # compared with the oracle's 50 sweeps from the same start
    specs = synth.batch_instances(512, 900)
    size = [int(np.prod(dm)) for dm, _ in specs]
    order = np.argsort(size)[::-1]
    pick = list(order[:4]) + list(order[100:500:100])
    As, x0s, exact = [], [], []
    for i in pick:
        dims, lam = specs[i]
        A = synth.device_normal(dims, 1000 + int(i), dev)
        vecs = synth.unit_vectors(dims, 3000 + int(i), "normal")
        outer = torch.ones((), dtype=torch.float64, device=dev)
        for v in vecs:
            outer = torch.tensordot(outer, torch.as_tensor(v, device=dev), dims=0)
        A.add_(outer.float(), alpha=lam)
        As.append(A)
        exact.append(A.cpu().numpy())
        x0s.append(synth.unit_vectors(dims, 5000 + int(i)))
    assert max(a.numel() for a in As) >= 200 ** 3
    xs = [tvc.pack_vectors(x0, dev) for x0 in x0s]
    sweeps = 50
    bp = B.prepare(As, xs, sweeps, tile_elems=1 << 20)
    B.run(bp)
    torch.cuda.synchronize()
    assert B.error_word(bp) == 0
    res = B.results(bp)
    for i, (A, x0) in enumerate(zip(exact, x0s)):
        ref = H.hopm(A, x0, sweeps=sweeps, form="kron", workers=16)
        got = np.split(host(xs[i]), np.cumsum(A.shape)[:-1])
        assert abs(res[i].lam - ref.lam) < 2e-5 * ref.lam, (i, A.shape, res[i].lam, ref.lam)
        for g, r in zip(got, ref.xs):
            assert np.linalg.norm(g - r) < 2e-4, (i, A.shape, np.linalg.norm(g - r))
        assert res[i].sweeps == sweeps and res[i].status == 0
