"""Derivatives at the full 256^4 float32 size (2^32 elements, 17.2 GB),
where 64-bit element offsets are live in every backward kernel:
dx in every mode against the oracle's adjoint computed mode-0 slab by slab
from the exact host copy of the device bytes, dA on sampled entries
bitwise, and the gradient through 10 unrolled HOPM sweeps: its forward
trajectory sweep by sweep against the float64 oracle, and the homogeneity
identities that hold at any size."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import grad as G
from oracle import hopm as H
from oracle import tvc as O
from paper_2501_03121_amd import autograd as AG
from paper_2501_03121_amd import synth
from _util import host

pytestmark = pytest.mark.gpu

DIMS = (256, 256, 256, 256)
N = 256 ** 4


@pytest.fixture(scope="module")
def big(dev):
    A = synth.device_normal(DIMS, 500, dev)
    Ah = A.cpu().numpy()
    yield A, Ah
    del A
    torch.cuda.empty_cache()


def _grad_x_by_slabs(Ah, gh, k):
    # dx = A contracted with g over every mode but k, summed over the
    # mode-0 slabs of A (each slab's adjoint from the oracle, in float64)
    if k == 0:
        return np.array([G.tvc_grad_x(Ah[m:m + 1], gh[None], 0)[0] for m in range(DIMS[0])])
    out = np.zeros(DIMS[k])
    for i in range(DIMS[0]):
        out += G.tvc_grad_x(Ah[i].astype(np.float64), gh[i], k - 1)
    return out


@pytest.mark.timeout(1200)
def test_backward_x_256_4_every_mode(dev, big):
    A, Ah = big
    assert A.numel() == N == 2 ** 32
    for k in range(4):
        g = synth.device_normal((N // DIMS[k],), 600 + k, dev)
        dx = host(tvc.backward_x(A, g, k))
        gh = g.cpu().numpy().reshape(O.output_dims(DIMS, k))
        ref = _grad_x_by_slabs(Ah, gh, k)
        assert O.rel_err(dx, ref) < 1e-5, k
        # every entry, not only the norm
        assert np.max(np.abs(dx - ref)) <= 1e-5 * np.sqrt(np.mean(ref ** 2)), k
        del g


@pytest.mark.timeout(600)
def test_backward_A_256_4_sampled_bitwise(dev):
    S = 65536
    for k in range(4):
        u, n, v = O.matricized_dims(DIMS, k)
        g = synth.device_normal((u * v,), 700 + k, dev)
        x = torch.from_numpy(synth.uniform(n, 710 + k).astype(np.float32)).to(dev)
        dA = tvc.backward_A(g, x, k, DIMS)
        rng = synth.rng(720 + k)
        l, m, r = rng.integers(0, u, S), rng.integers(0, n, S), rng.integers(0, v, S)
        l[:2], m[:2], r[:2] = [0, u - 1], [0, n - 1], [0, v - 1]
        li, mi, ri = (torch.from_numpy(t).to(dev) for t in (l, m, r))
        got = dA.view(u, n, v)[li, mi, ri].cpu().numpy()
        gs = g.view(u, v)[li, ri].cpu().numpy().astype(np.float64)
        full = G.tvc_grad_A(gs.reshape(S, 1), host(x), 1, (S, n, 1))
        ref = full[np.arange(S), m, 0].astype(np.float32)
        np.testing.assert_array_equal(got, ref)
        del dA, g


K = 10


def _recorded_forward(A, x0, dev):
    # the forward sweeps the autograd function records, one at a time
    x = tvc.pack_vectors(x0, dev)
    norms = torch.empty(K * 4, dtype=torch.float64, device=dev)
    traj = []
    for i in range(K):
        tvc.hopm_iterate_record(A, x, 1, norms[4 * i:4 * i + 4])
        traj.append(host(x).copy())
    return traj, host(norms)


@pytest.mark.timeout(900)
def test_unrolled_hopm_256_4_forward_trajectory(dev, big):
    A, Ah = big
    x0 = synth.unit_vectors(DIMS, 800)
    traj, nr = _recorded_forward(A, x0, dev)
    xs = [np.asarray(v) for v in x0]
    for i in range(K):
        o = H.hopm(Ah, xs, sweeps=1, form="kron", workers=16)
        xs = o.xs
        got = np.split(traj[i], np.cumsum(DIMS)[:-1])
        for j in range(4):
            assert np.linalg.norm(got[j] - xs[j]) < 1e-5, (i, j)
        np.testing.assert_allclose(nr[4 * i:4 * i + 4], o.norms, rtol=1e-5)


@pytest.mark.timeout(900)
def test_unrolled_hopm_256_4_gradient_identities(dev, big):
    A, _ = big
    x0 = synth.unit_vectors(DIMS, 800)
    traj, nr = _recorded_forward(A, x0, dev)
    # the differentiable K-sweep HOPM: same forward, then the reverse pass
    Ar = A.requires_grad_(True)
    xt = [torch.from_numpy(v).to(dev).requires_grad_(True) for v in x0]
    out = AG.hopm(Ar, K, *xt)
    lam = out[0]
    assert float(lam) == float(nr[-1])
    assert torch.equal(torch.cat([t.detach() for t in out[1:]]), torch.from_numpy(traj[-1]).to(dev))
    lam.backward()
    # Euler: lambda(cA) = c lambda(A), so <d lambda / dA, A> = lambda
    lhs = sum(float((Ar.grad[i].double() * A.detach()[i].double()).sum()) for i in range(DIMS[0]))
    assert abs(lhs - float(lam)) < 1e-4 * float(lam)
    # the first sweep recomputes x_0 before reading it: no gradient to it;
    # the others enter only through their directions: <d lambda / dx_m, x_m> = 0
    assert float(xt[0].grad.abs().max()) <= 1e-12 * float(lam)
    for m in range(1, 4):
        gm = xt[m].grad
        assert float(gm.norm()) > 0
        assert abs(float((gm * xt[m].detach()).sum())) <= 1e-5 * float(gm.norm()), m
    A.requires_grad_(False)
    A.grad = None
