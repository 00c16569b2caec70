"""Parity of the HIP HOPM (hopm_iterate / hopm_solve through the C ABI) with
the float64 canonical HOPM oracle from the same initial vectors."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import hopm as H
from oracle import quant as Q
from oracle import tvc as O
from paper_2501_03121_amd import synth
from _util import host, stored_tensor

pytestmark = pytest.mark.gpu


def run_sweeps(A, x0, sweeps, dev, scale=None):
    x = tvc.pack_vectors(x0, dev)
    traj = []
    for _ in range(sweeps):
        st = tvc.hopm_iterate(A, x, 1, scale=scale)
        r = tvc.read_stats(st)
        traj.append((host(x).copy(), r))
    return traj


def check_traj(traj, exact, x0, tol_vec, tol_lam):
    dims = exact.shape
    ref = H.hopm(exact, x0, sweeps=len(traj))
    xs = [np.asarray(v) for v in x0]
    for i, (xg, r) in enumerate(traj):
        o = H.hopm(exact, xs, sweeps=1)
        xs = o.xs
        got = np.split(xg, np.cumsum(dims)[:-1])
        for j in range(len(dims)):
            assert np.linalg.norm(got[j] - xs[j]) <= tol_vec, (i, j, np.linalg.norm(got[j] - xs[j]))
        assert abs(r.lam - o.lam) <= tol_lam * abs(o.lam), (i, r.lam, o.lam)
        assert abs(r.delta - o.deltas[0]) <= tol_vec + 1e-3 * o.deltas[0]
        assert r.sweeps == 1 and r.status == 0
    return ref


def test_tiny_planted_fp64_20_sweeps(dev):
    dims = (64, 64, 64)
    A, a = synth.planted_rank1(dims, 5.0, 0.01, 100)
    x0 = synth.unit_vectors(dims, 103)
    At = torch.from_numpy(A).to(dev)
    traj = run_sweeps(At, x0, 20, dev)
    check_traj(traj, A, x0, 1e-12, 1e-12)
    xg = np.split(traj[-1][0], [64, 128])
    for x, v in zip(xg, a):
        assert abs(np.dot(x, v)) > 0.9999
    assert abs(traj[-1][1].lam - 5.0) < 0.05


@pytest.mark.parametrize("dims", [(40, 33), (9, 17, 5), (6, 5, 7, 4), (4, 3, 5, 2, 6), (3, 4, 2, 3, 5, 2),
                                  (128, 1, 96), (1, 64, 64)])
@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_trajectory_parity(dev, dims, fmt):
    A, _, exact = stored_tensor(dims, fmt, 7, dev, kind="normal")
    x0 = synth.unit_vectors(dims, 8)
    traj = run_sweeps(A, x0, 4, dev)
    tol = 1e-11 if fmt == "f64" else 2e-5
    check_traj(traj, exact, x0, tol, tol)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("dims", [(33, 40, 17), (12, 9, 10, 11)])
def test_low_precision_parity_on_stored_values(dev, fmt, dims):
    A, S, exact = stored_tensor(dims, fmt, 9, dev, kind="normal")
    x0 = synth.unit_vectors(dims, 10)
    traj = run_sweeps(A, x0, 3, dev, scale=S)
    check_traj(traj, exact, x0, 2e-5, 2e-5)


@pytest.mark.parametrize("dims", [(30, 20, 10), (8, 9, 7, 6), (5, 6, 4, 3, 5)])
def test_exact_rank1_one_sweep(dev, dims):
    a = synth.unit_vectors(dims, 1)
    T = np.ones(())
    for v in a:
        T = np.multiply.outer(T, v)
    At = torch.from_numpy(3.25 * T).to(dev)
    x = tvc.pack_vectors(synth.unit_vectors(dims, 2), dev)
    r = tvc.read_stats(tvc.hopm_iterate(At, x, 1))
    assert abs(r.lam - 3.25) < 1e-12 * 3.25
    for g, v in zip(np.split(host(x), np.cumsum(dims)[:-1]), a):
        assert abs(abs(np.dot(g, v)) - 1) < 1e-12


def test_matrix_case_matches_svd(dev):
    A = synth.normal((300, 200), 3)
    A += 40 * np.outer(synth.unit_vectors([300], 4)[0], synth.unit_vectors([200], 5)[0])
    x = tvc.pack_vectors(synth.unit_vectors((300, 200), 6), dev)
    r = tvc.hopm_solve(torch.from_numpy(A).to(dev), x, tol=1e-12, max_sweeps=500)
    assert r.status == 0
    U, S, Vt = np.linalg.svd(A)
    assert abs(r.lam - S[0]) < 1e-10 * S[0]
    g = host(x)
    assert abs(abs(np.dot(g[:300], U[:, 0])) - 1) < 1e-9
    assert abs(abs(np.dot(g[300:], Vt[0])) - 1) < 1e-9


def test_solve_converges_and_reports(dev):
    dims = (48, 40, 36)
    A, a = synth.planted_rank1(dims, 6.0, 0.02, 50, noise_kind="normal")
    x0 = synth.unit_vectors(dims, 53)
    At = torch.from_numpy(A.astype(np.float32)).to(dev)
    x = tvc.pack_vectors(x0, dev)
    r = tvc.hopm_solve(At, x, tol=1e-6, max_sweeps=200, check_every=2)
    assert r.status == 0 and r.delta < 1e-6 and r.sweeps % 2 == 0
    ref = H.hopm(At.cpu().double().numpy(), x0, tol=1e-6, max_sweeps=200)
    assert abs(r.lam - ref.lam) < 1e-5 * ref.lam
    x = tvc.pack_vectors(x0, dev)
    r2 = tvc.hopm_solve(At, x, tol=0.0, max_sweeps=3)
    assert r2.status == 7 and r2.sweeps == 3     # TVC_ENOTCONVERGED


def test_degenerate_zero_tensor(dev):
    At = torch.zeros((5, 6, 7), dtype=torch.float32, device=dev)
    x0 = synth.unit_vectors((5, 6, 7), 0)
    x = tvc.pack_vectors(x0, dev)
    r = tvc.read_stats(tvc.hopm_iterate(At, x, 2))
    assert r.status == 6            # TVC_EDEGENERATE
    np.testing.assert_array_equal(host(x), np.concatenate(x0))   # vectors unchanged
    with pytest.raises(tvc.TvcError):
        tvc.hopm_solve(At, x, tol=1e-6, max_sweeps=5)


def test_bf16_with_fp32_refinement(dev):
    # the refinement runs to tol on the float32 data: its stopping test gives
    # the status, and lambda then matches the float64 oracle to float32 level
    dims = (40, 36, 32)
    A, a = synth.planted_rank1(dims, 8.0, 0.05, 60, noise_kind="normal", vec_kind="normal")
    A32 = torch.from_numpy(A.astype(np.float32)).to(dev)
    Ab, _ = tvc.quantize(A32, "bf16")
    x0 = synth.unit_vectors(dims, 63)
    x = tvc.pack_vectors(x0, dev)
    r = tvc.hopm_solve(Ab, x, tol=1e-6, max_sweeps=300, A_refine=A32, refine_sweeps=100)
    assert r.status == 0 and r.delta < 1e-6 and 1 <= r.refine_sweeps < 100
    ref = H.hopm(A32.cpu().double().numpy(), x0, tol=1e-10, max_sweeps=2000)
    assert abs(r.lam - ref.lam) <= 1e-5 * ref.lam
    got = np.split(host(x), np.cumsum(dims)[:-1])
    for g, e in zip(got, ref.xs):
        assert np.linalg.norm(g - e) < 1e-4


def test_refinement_status_is_the_last_stage(dev):
    dims = (40, 36, 32)
    A, a = synth.planted_rank1(dims, 8.0, 0.05, 60, noise_kind="normal", vec_kind="normal")
    A32 = torch.from_numpy(A.astype(np.float32)).to(dev)
    Ab, _ = tvc.quantize(A32, "bf16")
    x0 = synth.unit_vectors(dims, 63)
    # a refinement cut off at one sweep has not met tol: not converged, even
    # though the bf16 stage converged
    x = tvc.pack_vectors(x0, dev)
    r = tvc.hopm_solve(Ab, x, tol=1e-6, max_sweeps=300, A_refine=A32, refine_sweeps=1)
    assert r.status == 7 and r.refine_sweeps == 1 and r.delta >= 1e-6
    # a bf16 stage cut off at its cap, then a refinement that converges: ok
    x = tvc.pack_vectors(x0, dev)
    r = tvc.hopm_solve(Ab, x, tol=1e-6, max_sweeps=2, A_refine=A32, refine_sweeps=200)
    assert r.status == 0 and r.sweeps == 2 and r.delta < 1e-6
    # refine_sweeps = 0: no refinement, the first stage decides
    x = tvc.pack_vectors(x0, dev)
    r = tvc.hopm_solve(Ab, x, tol=1e-6, max_sweeps=2, A_refine=A32, refine_sweeps=0)
    assert r.status == 7 and r.refine_sweeps == 0
