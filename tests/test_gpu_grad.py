"""Derivatives through the C ABI: the contraction's backward kernels, the
leave-one-out contraction, the rank-R update and the reverse pass through
unrolled HOPM sweeps, against the float64 oracle and finite differences."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import grad as G
from oracle import hopm as H
from oracle import tvc as O
from paper_2501_03121_amd import autograd as AG
from paper_2501_03121_amd import synth
from _util import TOL, host, stored_tensor

pytestmark = pytest.mark.gpu

SHAPES = [(7, 13, 5), (64, 64, 64), (3, 1, 4, 9), (17, 19, 23, 3), (5, 2, 70001), (3, 50000, 4),
          (2, 3, 4, 5, 6, 7), (1000003,)]


@pytest.mark.parametrize("fmt", ["f64", "f32", "bf16", "e4m3"])
@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_backward_x_all_modes(dev, fmt, dims):
    A, S, exact = stored_tensor(dims, fmt, 3, dev)
    acc = torch.float64 if fmt == "f64" else torch.float32
    for k in range(len(dims)):
        gh = synth.uniform(O.output_dims(dims, k), 40 + k)
        gt = torch.from_numpy(gh).to(acc).to(dev).reshape(-1)
        dx = tvc.backward_x(A, gt, k, scale=S)
        ref = G.tvc_grad_x(exact, host(gt).reshape(O.output_dims(dims, k)), k)
        assert O.rel_err(host(dx), ref) <= TOL[fmt], (fmt, dims, k)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("dims", SHAPES[:7], ids=lambda d: "x".join(map(str, d)))
def test_backward_A_all_modes(dev, fmt, dims):
    acc = torch.float64 if fmt == "f64" else torch.float32
    for k in range(len(dims)):
        gh = synth.uniform(O.output_dims(dims, k), 50 + k)
        xh = synth.uniform(dims[k], 60 + k)
        g = torch.from_numpy(gh).to(acc).to(dev).reshape(-1)
        x = torch.from_numpy(xh).to(acc).to(dev)
        dA = tvc.backward_A(g, x, k, dims)
        ref = G.tvc_grad_A(host(g).reshape(O.output_dims(dims, k)), host(x), k, dims)
        np.testing.assert_array_equal(host(dA), ref.astype(np.float32 if fmt == "f32" else np.float64))
        prev = torch.from_numpy(synth.uniform(dims, 70)).to(acc).to(dev)
        out = prev.clone()
        tvc.backward_A(g, x, k, dims, alpha=0.5, beta=-2.0, out=out)
        assert O.rel_err(host(out), 0.5 * ref - 2.0 * host(prev)) < (1e-12 if fmt == "f64" else 1e-6)


def test_adjoint_identity_through_autograd(dev):
    dims = (12, 40, 9, 6)
    A, _, exact = stored_tensor(dims, "f64", 5, dev)
    for k in range(4):
        x = torch.from_numpy(synth.uniform(dims[k], 80 + k)).to(dev).requires_grad_(True)
        Ar = A.clone().requires_grad_(True)
        y = AG.tvc(Ar, x, k)
        g = torch.from_numpy(synth.uniform(tuple(y.shape), 90 + k)).to(dev)
        (y * g).sum().backward()
        np.testing.assert_allclose(host(x.grad), G.tvc_grad_x(exact, host(g), k), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(host(Ar.grad), G.tvc_grad_A(host(g), host(x.detach()), k, dims),
                                   rtol=1e-15, atol=0)


@pytest.mark.parametrize("fmt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("dims", [(9, 11), (7, 13, 5), (5, 6, 4, 3), (4, 3, 5, 2, 3), (3, 4, 2, 3, 2, 3)])
def test_leave_one_out(dev, fmt, dims):
    A, S, exact = stored_tensor(dims, fmt, 6, dev, kind="normal")
    vs = [synth.uniform(n, 100 + i) for i, n in enumerate(dims)]
    v = tvc.pack_vectors(vs, dev)
    out = tvc.leave_one_out(A, v, scale=S)
    got = np.split(host(out), np.cumsum(dims)[:-1])
    for m in range(len(dims)):
        ref = H.leave_one_out(exact, vs, m)
        assert O.rel_err(got[m], ref) <= TOL[fmt] * 2, (fmt, dims, m)
    part = tvc.leave_one_out(A, v, modes=[len(dims) - 1], scale=S)
    assert np.all(host(part)[: sum(dims[:-1])] == 0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("dims,R", [((6, 7, 5), 3), ((16, 16, 16, 16), 41), ((3, 300), 2), ((5, 4, 3, 2, 70), 17)])
def test_rank_update(dev, dtype, dims, R):
    fh = synth.normal((R, sum(dims)), 7)
    ch = synth.normal(R, 8)
    Ah = synth.normal(dims, 9)
    ref = -1.5 * Ah
    for r in range(R):
        vecs = np.split(fh[r], np.cumsum(dims)[:-1])
        ref = ref + ch[r] * G.outer(vecs)
    A = torch.from_numpy(Ah).to(dtype).to(dev)
    D = tvc.rank_update(dims, torch.from_numpy(fh).to(dev), torch.from_numpy(ch).to(dev), A=A, alpha=-1.5,
                        dtype=dtype)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert O.rel_err(host(D), ref) < tol
    D2 = A.clone()
    tvc.rank_update(dims, torch.from_numpy(fh).to(dev), torch.from_numpy(ch).to(dev), A=D2, alpha=-1.5, out=D2)
    assert O.rel_err(host(D2), ref) < tol


@pytest.mark.parametrize("dims,K", [((5, 4, 3), 4), ((12, 12, 12, 12), 10), ((6, 5, 4, 3, 2), 3), ((20, 30), 5),
                                    ((4, 3, 2, 3, 2, 3, 2), 3), ((2, 3, 2, 2, 3, 2, 2, 3, 2), 2)])
def test_unrolled_hopm_grad_fp64_vs_oracle(dev, dims, K):
    Ah = synth.normal(dims, 11)
    x0 = synth.unit_vectors(dims, 12)
    L_ref, gA_ref, gx_ref = G.hopm_loss_and_grad(Ah, x0, K)
    A = torch.from_numpy(Ah).to(dev).requires_grad_(True)
    xs = [torch.from_numpy(v).to(dev).requires_grad_(True) for v in x0]
    L = AG.rank1_loss(A, K, *xs)
    L.backward()
    assert abs(float(L) - L_ref) < 1e-10 * abs(L_ref)
    assert O.rel_err(host(A.grad), gA_ref) < 1e-10
    for g, r in zip(xs, gx_ref):
        assert np.linalg.norm(host(g.grad) - r) < 1e-9 * max(1.0, np.linalg.norm(r))


def test_unrolled_hopm_grad_fd_12_4(dev):
    # finite differences of the GPU loss itself, float64, 12^4, K = 10
    dims, K = (12, 12, 12, 12), 10
    Ah = synth.normal(dims, 13)
    x0 = [torch.from_numpy(v).to(dev) for v in synth.unit_vectors(dims, 14)]
    A = torch.from_numpy(Ah).to(dev).requires_grad_(True)
    L = AG.rank1_loss(A, K, *x0)
    L.backward()
    h = 1e-5
    for t in range(3):
        E = torch.from_numpy(synth.normal(dims, 200 + t)).to(dev)
        with torch.no_grad():
            lp = float(AG.rank1_loss(A + h * E, K, *x0))
            lm = float(AG.rank1_loss(A - h * E, K, *x0))
        fd = (lp - lm) / (2 * h)
        an = float((A.grad * E).sum())
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("dims", [(48, 40, 32, 24), (16, 16, 16, 16, 16)])
def test_unrolled_hopm_grad_fp32_euler_identity(dev, dims):
    # the sweeps only see directions: lambda(cA) = c lambda(A) for c > 0, so
    # <d lambda / dA, A> = lambda (Euler), at any size
    K = 10
    A = synth.device_normal(dims, 15, dev).requires_grad_(True)
    x0 = [torch.from_numpy(v).to(dev) for v in synth.unit_vectors(dims, 16)]
    lam = AG.hopm(A, K, *x0)[0]
    lam.backward()
    lhs = float((A.grad.double() * A.detach().double()).sum())
    assert abs(lhs - float(lam)) < 1e-4 * float(lam)
