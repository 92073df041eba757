"""Pins of the oracle's 1D PPM remap (the core of one shear, Section 2.1),
against facts fixed by the mathematics rather than by re-typing the formulas:
exactness on polynomials, exact shifts, conservation, positivity and the
defining property of the monotonicity limiter."""
import numpy as np
import pytest

import oracle

EPS = np.finfo(np.float64).eps
L = 16
UPD = slice(3, L - 3)


def cell_avg_poly(coefs, lo, hi):
    """Exact average of sum coefs[k] x^k over [lo, hi]."""
    P = np.polynomial.polynomial.Polynomial(coefs).integ()
    return (P(hi) - P(lo)) / (hi - lo)


@pytest.mark.parametrize("c", [-1.0, -0.7, -0.25, 0.0, 0.3, 0.5, 1.0])
def test_constant_state_is_preserved_bitwise(c):
    a = np.full(L, 3.7e-9)
    r = oracle.ppm_line(a, c)
    assert np.array_equal(r["out"], a)


def test_zero_courant_is_identity_bitwise():
    rng = np.random.default_rng(1)
    a = rng.uniform(0.0, 1.0, L)
    assert np.array_equal(oracle.ppm_line(a, 0.0)["out"], a)


@pytest.mark.parametrize("c,shift", [(1.0, 1), (-1.0, -1)])
def test_unit_courant_is_an_exact_shift(c, shift):
    rng = np.random.default_rng(2)
    for _ in range(20):
        a = rng.uniform(0.0, 1.0, L) * rng.choice([1.0, 0.0], L, p=[0.8, 0.2])
        out = oracle.ppm_line(a, c)["out"]
        want = np.roll(a, shift)
        assert np.max(np.abs(out[UPD] - want[UPD])) <= 2 * EPS * np.max(np.abs(a))


@pytest.mark.parametrize("coefs", [(1.0, 0.3, 0.01), (5.0, -0.4, -0.02), (2.0, 0.05, 0.0)])
@pytest.mark.parametrize("c", [-0.9, -0.5, -0.1, 0.2, 0.5, 1.0])
def test_quadratic_is_remapped_exactly(coefs, c):
    """Cell averages of a quadratic without an extremum on the line: PPM
    reconstructs the quadratic exactly, so the remap must return the exact
    averages of the profile shifted by c cells."""
    x = np.arange(L, dtype=np.float64)
    a = cell_avg_poly(coefs, x, x + 1)
    out = oracle.ppm_line(a, c)["out"]
    want = cell_avg_poly(coefs, x - c, x + 1 - c)
    assert np.max(np.abs(out[UPD] - want[UPD])) <= 50 * EPS * np.max(np.abs(a))


def test_cubic_face_values_are_point_values():
    """The fourth-order face interpolation is exact on cubics."""
    coefs = (1.0, 0.8, 0.03, 0.001)
    x = np.arange(L, dtype=np.float64)
    a = cell_avg_poly(coefs, x, x + 1)
    face = oracle.ppm_line(a, 0.5)["face"]
    pv = np.polynomial.polynomial.polyval(x + 1, coefs)  # value at face i+1/2 = x_{i}+1
    i = np.arange(2, L - 4)  # faces whose 4-cell stencils are inside the line
    assert np.max(np.abs(face[i] - pv[i])) <= 20 * EPS * np.max(np.abs(a))


def test_step_profile_hand_worked():
    """Step 0 -> 1 between cells 7 and 8, c = 1/2.  Every slope is zero
    (no cell is strictly monotone between its neighbours), the face between
    the plateaus is 1/2, both cells at the step are extrema of their
    stencils and are flattened: cell 8 sends half its content on and receives
    nothing, so averages become ..., 0, 0.5, 1, ...  (worked by hand)."""
    a = np.array([0.0] * 8 + [1.0] * 8)
    r = oracle.ppm_line(a, 0.5)
    assert r["face"][7] == 0.5
    assert r["al"][7] == r["ar"][7] == 0.0
    assert r["al"][8] == r["ar"][8] == 1.0
    want = a.copy()
    want[8] = 0.5
    assert np.array_equal(r["out"][UPD], want[UPD])


def test_limited_profile_has_no_interior_extremum():
    """CW84's limiter: afterwards each cell's parabola is monotone on the cell
    (|a6| <= |aR - aL|) or flat, and where the raw parabola had an interior
    extremum in a cell that is not itself an extremum, the extremum is moved
    exactly onto a cell edge (|a6| = |aR - aL|)."""
    rng = np.random.default_rng(3)
    n_moved = 0
    for _ in range(200):
        a = np.cumsum(rng.uniform(-0.2, 1.0, L)) + rng.normal(0, 0.3, L)
        r = oracle.ppm_line(a, 0.4)
        for i in range(2, L - 2):
            al, ar, a6 = r["al"][i], r["ar"][i], r["a6"][i]
            dA = ar - al
            scale = max(abs(a[i]), abs(al), abs(ar), 1e-300)
            if al == ar == a[i]:
                continue
            assert abs(a6) <= abs(dA) + 64 * EPS * scale
            # raw faces
            l0, r0 = r["face"][i - 1], r["face"][i]
            raw6 = 6.0 * (a[i] - 0.5 * (l0 + r0))
            if (r0 - a[i]) * (a[i] - l0) > 0 and abs(raw6) > abs(r0 - l0) * (1 + 1e-9):
                assert abs(abs(a6) - abs(dA)) <= 64 * EPS * scale
                n_moved += 1
    assert n_moved > 20


def test_limiter_flattens_local_extrema():
    a = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 2.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    r = oracle.ppm_line(a, 0.5)
    assert r["al"][7] == r["ar"][7] == 2.0
    assert r["a6"][7] == 0.0


@pytest.mark.parametrize("c", [-1.0, -0.6, -0.2, 0.2, 0.6, 1.0])
def test_positivity_and_zero_cells(c):
    """Nonnegative data stays nonnegative, and a cell holding zero next to
    nonnegative neighbours sends no flux in either direction (this is what
    lets absent velocity blocks read as zero)."""
    rng = np.random.default_rng(4)
    for _ in range(200):
        a = rng.uniform(0.0, 1.0, L) * (rng.uniform(size=L) < 0.6)
        r = oracle.ppm_line(a, c)
        assert np.all(r["out"][UPD] >= -4 * EPS * a.max())
        for i in range(2, L - 3):
            if c > 0 and a[i] == 0.0:
                assert r["flux"][i] == 0.0
            if c < 0 and a[i + 1] == 0.0:
                assert r["flux"][i] == 0.0


@pytest.mark.parametrize("c", [-0.8, -0.3, 0.45, 0.9])
def test_line_telescopes(c):
    rng = np.random.default_rng(5)
    a = rng.uniform(0.0, 1.0, L)
    r = oracle.ppm_line(a, c)
    lhs = r["out"][UPD].sum() - a[UPD].sum()
    rhs = r["flux"][2] - r["flux"][L - 4]
    assert abs(lhs - rhs) <= 32 * EPS * a.sum()


def _periodic_advect(n, c, periods=1):
    x = (np.arange(n) + 0.5) / n
    # exact cell averages of 1 + 0.5 sin(2 pi x)
    lo, hi = np.arange(n) / n, (np.arange(n) + 1) / n
    u0 = 1.0 + 0.5 * (np.cos(2 * np.pi * lo) - np.cos(2 * np.pi * hi)) / (2 * np.pi / n)
    u = u0.copy()
    steps = int(round(n * periods / abs(c)))
    for _ in range(steps):
        line = np.concatenate([u[-3:], u, u[:3]])
        out = oracle.ppm_line(line, c)["out"]
        u = out[3:-3]
    return np.mean(np.abs(u - u0)), x


def test_convergence_order_on_smooth_periodic_data():
    e1, _ = _periodic_advect(32, 0.5)
    e2, _ = _periodic_advect(64, 0.5)
    e3, _ = _periodic_advect(128, 0.5)
    assert e2 < e1 and e3 < e2
    assert np.log2(e2 / e3) >= 1.8
