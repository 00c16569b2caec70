"""Pins of the derivative oracle: adjoint identities, brute force, and
central finite differences in float64 through unrolled HOPM sweeps.
CPU only."""
import numpy as np
import pytest

from oracle import grad as G
from oracle import tvc as O
from paper_2501_03121_amd import synth


@pytest.mark.parametrize("dims", [(4, 3, 5), (2, 3, 2, 4), (6, 5)])
def test_adjoint_identity(dims):
    A = synth.normal(dims, 1)
    for k, n in enumerate(dims):
        x = synth.normal(n, 2)
        g = synth.normal(O.output_dims(dims, k), 3)
        lhs = float(np.sum(O.tvc(A, x, k) * g))
        assert abs(lhs - float(np.sum(A * G.tvc_grad_A(g, x, k, dims)))) < 1e-12 * (1 + abs(lhs))
        assert abs(lhs - float(np.dot(x, G.tvc_grad_x(A, g, k)))) < 1e-12 * (1 + abs(lhs))


def test_grad_x_brute_force():
    dims = (3, 4, 2)
    A = synth.integers(dims, 4, -9, 9)
    for k, n in enumerate(dims):
        g = synth.integers(O.output_dims(dims, k), 5, -9, 9)
        ref = np.zeros(n)
        for m in range(n):
            e = np.zeros(n)
            e[m] = 1.0
            ref[m] = np.sum(O.tvc_loops(A, e, k) * g)
        assert np.array_equal(G.tvc_grad_x(A, g, k), ref)


def test_loss_identity():
    dims = (5, 4, 3, 4)
    A = synth.normal(dims, 6)
    x0 = synth.unit_vectors(dims, 7)
    L, _, _ = G.hopm_loss_and_grad(A, x0, 3)
    assert abs(L - G.hopm_loss(A, x0, 3)) < 1e-10 * abs(L)


@pytest.mark.parametrize("dims,K", [((5, 4, 3), 4), ((4, 3, 4, 3), 3), ((12, 12, 12, 12), 10)])
def test_unrolled_hopm_grad_vs_finite_differences(dims, K):
    A = synth.normal(dims, 8)
    x0 = synth.unit_vectors(dims, 9)
    _, gA, _ = G.hopm_loss_and_grad(A, x0, K)
    h = 1e-5
    for t in range(3):
        E = synth.normal(dims, 100 + t)
        fd = (G.hopm_loss(A + h * E, x0, K) - G.hopm_loss(A - h * E, x0, K)) / (2 * h)
        an = float(np.sum(gA * E))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (fd, an)


def test_init_vector_grad_vs_finite_differences():
    dims = (4, 5, 3)
    A = synth.normal(dims, 10)
    x0 = synth.unit_vectors(dims, 11)
    _, _, gx = G.hopm_loss_and_grad(A, x0, 3)
    h = 1e-6
    for j in range(3):
        e = synth.normal(dims[j], 12 + j)
        xp = [v.copy() for v in x0]
        xm = [v.copy() for v in x0]
        xp[j] += h * e
        xm[j] -= h * e
        fd = (G.hopm_loss(A, xp, 3) - G.hopm_loss(A, xm, 3)) / (2 * h)
        assert abs(fd - float(np.dot(gx[j], e))) < 1e-6 * max(1.0, abs(fd))
