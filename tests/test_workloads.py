"""The seeded input generators: random streams, operators, sizes and spectra (CPU only)."""

import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _dense(rp, ci, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


def test_splitmix64_reference_outputs():
    # published outputs of the SplitMix64 reference generator
    assert list(W.splitmix64(0, 4)) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                        0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert list(W.splitmix64(1234567, 2)) == [6457827717110365317, 3203168211198807973]
    # counter-based: any window of the stream is the same as the full stream
    assert np.array_equal(W.splitmix64(7, 5, offset=10), W.splitmix64(7, 15)[10:])


def test_distributions():
    u = W.uniform(3, 200000, -1.0, 1.0)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.01
    g = W.normal(4, 200000)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01
    e = W.exponential(5, 200000, 50.0)
    assert abs(e.mean() - 0.02) < 0.0005


@pytest.mark.parametrize("dims", [(4, 5, 6), (7, 7, 7), (1, 3, 2)])
def test_stencil7_structure_and_spectrum(dims):
    rp, ci, v = W.stencil7_csr(*dims)
    a = _dense(rp, ci, v)
    assert rp[-1] == W.stencil7_nnz(*dims)
    assert np.array_equal(a, a.T)
    assert np.all(np.diag(a) == 6.0)
    for i in range(len(rp) - 1):  # columns sorted within each row
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)
    ev = np.linalg.eigvalsh(a / 6.0)
    lo, hi = W.stencil7_bounds(*dims)
    assert abs(ev[0] - lo) < 1e-13 and abs(ev[-1] - hi) < 1e-13


def test_stencil5_spectrum():
    rp, ci, v = W.stencil5_csr(9, 7)
    ev = np.linalg.eigvalsh(_dense(rp, ci, v) / 4.0)
    assert np.allclose(ev, W.stencil5_eigenvalues(9, 7), atol=1e-13)


def test_table2_lap1600_size():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table2_table6_sizes.txt")) if not l.startswith("#")]
    lap = [r for r in rows if r and r[0] == "Lap1600"][0]
    rp, _, _ = W.stencil5_csr(1598)
    assert len(rp) - 1 == int(lap[2])
    assert int(rp[-1]) == int(lap[3])


def test_table6_lap3d_sizes_and_condition():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table2_table6_sizes.txt")) if not l.startswith("#")]
    for r in [r for r in rows if r and r[0] == "lap3d"]:
        nx, n_printed, kappa_printed = int(r[1]), float(r[2]), float(r[4])
        m = nx - 1  # interior points per axis
        assert abs(m ** 3 - n_printed) <= 0.05 * n_printed
        lo, hi = W.stencil7_bounds(m)
        assert abs(hi / lo - kappa_printed) <= 0.01 * kappa_printed


def test_harmonic27_operator():
    kappa = W.harmonic27_kappa(5, 4, 3, seed=1)
    assert np.array_equal(kappa, kappa.astype(np.float32).astype(np.float64))
    rp, ci, v = W.harmonic27_csr(kappa)
    a = _dense(rp, ci, v)
    assert np.allclose(a, a.T, rtol=0, atol=1e-14 * np.abs(a).max())
    assert np.all(np.diag(a) > 0)
    assert np.linalg.eigvalsh(a)[0] > 0
    # interior cell: 27 entries; the diagonal is the sum of the 26 harmonic means
    i = 1 + 5 * (1 + 4 * 1)
    row = a[i]
    assert np.count_nonzero(row) == 27
    assert abs(row[i] + (row.sum() - row[i])) <= 1e-12 * row[i]
    # corner cell: 8 neighbours in-domain; 19 ghost terms of its own coefficient
    row0 = a[0]
    assert np.count_nonzero(row0) == 8
    assert abs(row0[0] - (-(row0.sum() - row0[0]) + 19 * kappa.ravel()[0])) <= 1e-12 * row0[0]


def test_lognormal_coefficients():
    kappa = W.harmonic27_kappa(40, seed=1)
    g = np.log(kappa) / 2.0
    assert abs(g.mean()) < 0.02 and abs(g.std() - 1.0) < 0.02


def test_q1_reference_stiffness_rigid_modes():
    k = W.q1_reference_stiffness(0.3)
    ev = np.linalg.eigvalsh(k)
    assert np.allclose(k, k.T, atol=1e-15)
    assert np.sum(np.abs(ev) < 1e-12) == 6 and ev.min() > -1e-12
    # translations are in the null space
    for c in range(3):
        t = np.zeros(24)
        t[c::3] = 1.0
        assert np.abs(k @ t).max() < 1e-12


@pytest.mark.parametrize("n_free", [2, 4, 6])
def test_elasticity_operator(n_free):
    rp, ci, v = W.elasticity_q1_csr(n_free, seed=2)
    assert len(rp) - 1 == 3 * n_free ** 3
    assert int(rp[-1]) == 9 * (3 * n_free - 2) ** 3
    a = _dense(rp, ci, v)
    assert np.allclose(a, a.T, atol=1e-14)
    assert np.linalg.eigvalsh(a)[0] > 0
    e = W.elasticity_q1_moduli(n_free, seed=2)
    assert e.min() >= 0.9 and e.max() <= 1.1


def test_rhs_from_solution():
    rp, ci, v = W.stencil7_csr(3)
    x = W.uniform(0, 27, -1.0, 1.0)
    assert np.allclose(W.rhs_from_solution(rp, ci, v, x), _dense(rp, ci, v) @ x, atol=1e-14)
