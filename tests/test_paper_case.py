"""Host helpers of the paper's homogenized anode case (Sec. 4.1, Eq. 40-42, Tables 1-2), pinned
to what the formulas fix: the two readings of Eq. 40 differ by exactly sqrt(2), every
diffusivity is symmetric, Eq. 40 scales as T^1.75 / p and Eq. 42 as sqrt(T / M), Eq. 41 reduces to
eps/tau D_ij without Knudsen resistance and to the mean Knudsen term without molecular
resistance, the feed keeps H2/H2O = 4:1, and tau_ref gives the paper's time step."""

import math

import pytest

from paper_1809_01600_amd import paper_case as pc

T, P = pc.TABLE2["T"], pc.TABLE2["p"]
PAIRS = ((0, 1), (0, 2), (1, 2))


def _f(i, j, reading="printed", T=T, p=P):
    (_, Mi, Vi), (_, Mj, Vj) = pc.TABLE1[i], pc.TABLE1[j]
    return pc.fuller(T, p, Mi, Mj, Vi, Vj, reading)


@pytest.mark.parametrize("i,j", PAIRS)
def test_fuller_readings_and_symmetry(i, j):
    assert _f(i, j, "printed") / _f(i, j, "mean") == pytest.approx(math.sqrt(2.0), rel=1e-14)
    assert _f(i, j) == pytest.approx(_f(j, i), rel=1e-15)
    with pytest.raises(ValueError):
        _f(i, j, "other")


def test_fuller_scaling_in_T_and_p():
    a = _f(0, 1, T=800.0, p=1.0e5)
    assert _f(0, 1, T=1600.0, p=1.0e5) / a == pytest.approx(2.0 ** 1.75, rel=1e-14)
    assert _f(0, 1, T=800.0, p=2.0e5) / a == pytest.approx(0.5, rel=1e-14)
    # the correlation is in cm^2/s with p in bar: at 1 bar, T = 1 K, sqrt(m) = 1 and unit volumes
    assert pc.fuller(1.0, 1.0e5, 2.0, 2.0, 1.0, 1.0, "printed") == pytest.approx(0.00143e-4 / 4.0, rel=1e-14)


def test_knudsen_scaling():
    d = pc.knudsen(2.6e-6, 1000.0, 2.0)
    assert pc.knudsen(2.6e-6, 4000.0, 2.0) / d == pytest.approx(2.0, rel=1e-14)
    assert pc.knudsen(2.6e-6, 1000.0, 8.0) / d == pytest.approx(0.5, rel=1e-14)
    assert pc.knudsen(5.2e-6, 1000.0, 2.0) / d == pytest.approx(2.0, rel=1e-14)
    # (d_p / 3) times the mean molecular speed sqrt(8 R T / (pi M))
    assert d == pytest.approx(2.6e-6 / 3.0 * math.sqrt(8.0 * 8.3145 * 1000.0 / (math.pi * 2.0e-3)), rel=1e-14)


def test_effective_limits_and_symmetry():
    eps, tau = 0.46, 4.5
    assert pc.effective(1e-4, 1e300, 1e300, eps, tau) == pytest.approx(eps / tau * 1e-4, rel=1e-12)
    assert pc.effective(1e300, 2e-3, 6e-4, eps, tau) == pytest.approx(eps / (2 * tau) * (2e-3 + 6e-4), rel=1e-12)
    assert pc.effective(1e-4, 2e-3, 6e-4, eps, tau) == pytest.approx(pc.effective(1e-4, 6e-4, 2e-3, eps, tau), rel=1e-15)
    D = pc.diffusivities("printed")
    for (i, j), d in zip(PAIRS, D):
        assert d < eps / tau * _f(i, j)  # Knudsen resistance only lowers it


def test_feed_and_time_step():
    for x in (0.8, 0.5, 0.2):
        X = pc.feed(x)
        assert X[0] == 4.0 * X[1] and abs(sum(X) - 1.0) < 1e-15 and X[2] >= 0.0
    assert pc.feed(0.8)[2] == 0.0
    with pytest.raises(ValueError):
        pc.feed(0.9)
    D = pc.diffusivities("mean")
    tau = pc.tau_ref_for(D)
    assert (tau - 0.5) * pc.DX ** 2 / (3.0 * max(D)) == pytest.approx(pc.DT, rel=1e-14)
    c = pc.make_case(0.4, 0.7, "mean")
    assert (c.nx, c.ny, c.nz, c.lattice, c.dx) == (100, 1000, 1, "D2Q9", 20e-6)
    assert (c.D12, c.D13, c.D23) == D and c.X_in == pc.feed(0.4) and c.solid is None


def test_overpotential_definition():
    assert pc.overpotential(T, (0.8, 0.2, 0.0), (0.8, 0.2)) == 0.0
    v = pc.overpotential(T, (0.8, 0.2, 0.0), (0.4, 0.6))
    assert v == pytest.approx(8.3145 * T / (2 * 96485.0) * math.log(0.8 * 0.6 / (0.4 * 0.2)), rel=1e-15)
