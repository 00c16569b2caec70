"""Jacobi HOPM (hopm_jacobi_iterate / hopm_jacobi_solve through the C ABI):
the one-pass sweep against the float64 oracle's Jacobi variant from the
same initial vectors, in every storage format, for orders 2-10, ragged and
full-size shapes."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import hopm as H
from paper_2501_03121_amd import synth
from _util import host, stored_tensor

pytestmark = pytest.mark.gpu


def run_jacobi(A, x0, sweeps, dev, scale=None):
    x = tvc.pack_vectors(x0, dev)
    out = []
    for _ in range(sweeps):
        r = tvc.read_stats(tvc.hopm_jacobi_iterate(A, x, 1, scale=scale))
        out.append((host(x).copy(), r))
    return out


def check(traj, exact, x0, tol, form="chain"):
    dims = exact.shape
    xs = [np.asarray(v) for v in x0]
    for i, (xg, r) in enumerate(traj):
        o = H.jacobi_hopm(exact, xs, sweeps=1, form=form, workers=16)
        got = np.split(xg, np.cumsum(dims)[:-1])
        for j in range(len(dims)):
            assert np.linalg.norm(got[j] - o.xs[j]) <= tol, (i, j, np.linalg.norm(got[j] - o.xs[j]))
        assert abs(r.lam - o.lam) <= tol * o.lam, (i, r.lam, o.lam)
        assert abs(r.delta - o.deltas[0]) <= tol + 1e-3 * o.deltas[0], (i, r.delta, o.deltas[0])
        assert r.sweeps == 1 and r.status == 0
        xs = o.xs


SHAPES = [(40, 33), (300, 7), (9, 17, 5), (33, 40, 17), (6, 5, 7, 4), (4, 3, 5, 2, 6), (3, 4, 2, 3, 5, 2),
          (3, 2, 5, 3, 2, 3, 7), (2, 3, 2, 2, 3, 2, 2, 5, 2, 3), (128, 1, 96), (2, 3, 1001), (5, 2, 4099),
          # W = A x_0 x_0 x_1 x_1 above 8192 values: read once as a matrix of its
          # halves (once; twice, the first half again; ragged odd halves)
          (4, 3, 20, 21, 22), (2, 2, 5, 2000, 3, 2), (3, 2, 9, 11, 13, 7),
          # size-1 modes in W: one-row matrices and one-value halves
          (4, 4, 1, 1, 9000), (2, 3, 1, 5000, 1, 3)]


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_jacobi_trajectory(dev, dims, fmt):
    A, _, exact = stored_tensor(dims, fmt, 31, dev, kind="normal")
    x0 = synth.unit_vectors(dims, 32)
    # float32: far from convergence on noise (delta ~ 1) a Jacobi step can
    # amplify the float32 rounding of the previous sweep more than a
    # Gauss-Seidel step does; 4 sweeps stay within 5e-5
    check(run_jacobi(A, x0, 4, dev), exact, x0, 1e-11 if fmt == "f64" else 5e-5)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("dims", [(33, 40, 17), (12, 9, 10, 11), (64, 48), (2, 4, 1000), (3, 2, 9, 11, 13, 7)])
def test_jacobi_narrow_formats_on_stored_values(dev, fmt, dims):
    A, S, exact = stored_tensor(dims, fmt, 33, dev, kind="normal")
    x0 = synth.unit_vectors(dims, 34)
    check(run_jacobi(A, x0, 3, dev, scale=S), exact, x0, 2e-5)


@pytest.mark.parametrize("dims", [(3, 2, 9, 11, 13, 7), (6, 5, 7, 4)], ids=lambda d: "x".join(map(str, d)))
def test_jacobi_sweeps_in_one_call_equal_single_calls(dev, dims):
    # each sweep reads the previous sweep's vectors from the mirror that the
    # last step of the sweep before refreshed
    A, _, _ = stored_tensor(dims, "f32", 35, dev, kind="normal")
    x0 = synth.unit_vectors(dims, 36)
    xa = tvc.pack_vectors(x0, dev)
    ra = tvc.read_stats(tvc.hopm_jacobi_iterate(A, xa, 3))
    xb = tvc.pack_vectors(x0, dev)
    for _ in range(3):
        rb = tvc.read_stats(tvc.hopm_jacobi_iterate(A, xb, 1))
    assert torch.equal(xa, xb)
    assert ra.lam == rb.lam and ra.delta == rb.delta and ra.sweeps == 3 and rb.sweeps == 1


@pytest.mark.parametrize("dims", [(30, 20, 10), (8, 9, 7, 6), (50, 40)])
def test_jacobi_exact_rank1(dev, dims):
    a = synth.unit_vectors(dims, 1)
    T = np.ones(())
    for v in a:
        T = np.multiply.outer(T, v)
    At = torch.from_numpy(3.25 * T).to(dev)
    x = tvc.pack_vectors(synth.unit_vectors(dims, 2), dev)
    tvc.hopm_jacobi_iterate(At, x, 1)
    r = tvc.read_stats(tvc.hopm_jacobi_iterate(At, x, 1))
    assert abs(r.lam - 3.25) < 1e-12 * 3.25 and r.delta < 1e-12
    for g, v in zip(np.split(host(x), np.cumsum(dims)[:-1]), a):
        assert abs(abs(np.dot(g, v)) - 1) < 1e-12


def test_jacobi_solve_reaches_gauss_seidel_fixed_point(dev):
    dims = (48, 40, 36)
    A, a = synth.planted_rank1(dims, 6.0, 0.02, 50, noise_kind="normal")
    At = torch.from_numpy(A.astype(np.float32)).to(dev)
    x0 = synth.unit_vectors(dims, 53)
    xj = tvc.pack_vectors(x0, dev)
    rj = tvc.hopm_jacobi_solve(At, xj, tol=1e-6, max_sweeps=500)
    assert rj.status == 0 and rj.delta < 1e-6
    xg = tvc.pack_vectors(x0, dev)
    rg = tvc.hopm_solve(At, xg, tol=1e-6, max_sweeps=500)
    assert abs(rj.lam - rg.lam) < 1e-5 * rg.lam
    for u, v in zip(np.split(host(xj), np.cumsum(dims)[:-1]), np.split(host(xg), np.cumsum(dims)[:-1])):
        assert abs(abs(np.dot(u, v)) - 1) < 1e-5
    x = tvc.pack_vectors(x0, dev)
    r = tvc.hopm_jacobi_solve(At, x, tol=0.0, max_sweeps=3)
    assert r.status == 7 and r.sweeps == 3


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dims", [(1024, 1024, 1024), (32, 32, 32, 32, 32, 32), (175, 175, 175, 175)],
                         ids=["1024^3", "32^6", "175^4"])
def test_jacobi_full_size_sweep(dev, dims):
    A, a = synth.device_planted(dims, 10.0, 0.1, 200, dev)
    x0 = synth.warm_start(a, 0.9, 400)
    traj = run_jacobi(A, x0, 2, dev)
    Ah = A.cpu().numpy()
    del A
    torch.cuda.empty_cache()
    check(traj, Ah, x0, 1e-5, form="kron")


# Tensors whose one-pass strips outnumber the waves of a 256-CU part (rows
# of more than 2^20 16-byte units, split as n0 n1 x the rest): the rows are
# then not split into chunks, and the tasks run in more than one round; the
# last unit of a row is ragged in all but the first.
@pytest.mark.timeout(600)
@pytest.mark.parametrize("fmt,dims", [("f32", (8, 8, 4200000)), ("f32", (8, 9, 2049, 2049)),
                                      ("f64", (8, 8, 4200000)), ("f64", (9, 9, 1451, 1451))],
                         ids=["f32-8x8x4200000", "f32-8x9x2049x2049", "f64-8x8x4200000", "f64-9x9x1451x1451"])
def test_jacobi_strips_beyond_one_round(dev, fmt, dims):
    A, a = synth.device_planted(dims, 10.0, 0.1, 200, dev, dtype=torch.float64 if fmt == "f64" else None)
    x0 = synth.warm_start(a, 0.9, 400)
    traj = run_jacobi(A, x0, 2, dev)
    Ah = A.cpu().numpy()
    del A
    torch.cuda.empty_cache()
    check(traj, Ah, x0, 1e-10 if fmt == "f64" else 1e-5, form="kron")
