"""Pins of the oracle's pointwise building blocks against exact identities of
the Hermite machinery (Sec. 2.2-2.3, Sec. 3.3).  These check properties --
moments of the constructed populations -- not a retyped copy of the formulas
that build them."""
import numpy as np
import pytest

import oracle

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
CS2 = 1.0 / 3.0
HXX = CX * CX - CS2
HYY = CY * CY - CS2
HXY = CX * CY
HXXY = HXX * CY
HXYY = HYY * CX
HXXYY = HXX * HYY
HXXX = CX ** 3 - 3 * CS2 * CX

rng = np.random.default_rng(1234)
STATES = [(rng.uniform(0.5, 2.0), rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6),
           rng.uniform(0.1, 1.5)) for _ in range(12)]


@pytest.mark.parametrize("rho,ux,uy,th", STATES)
def test_feq_moments(rho, ux, uy, th):
    """Sum f = rho, sum c f = rho u, sum c c f = rho u u + p I with
    p = rho c_s^2 theta (Eqs. zero/first moment, Eq. perfect gas), and the
    third/fourth basis moments equal the equilibrium coefficients of
    Eqs. (a3)-(a4) for the supported tuples xxy, yyx, xxyy (Sec. 2.3)."""
    f = oracle.feq(rho, ux, uy, th)
    p = rho * CS2 * th
    tol = 1e-14
    assert f.sum() == pytest.approx(rho, rel=tol, abs=tol)
    assert (CX * f).sum() == pytest.approx(rho * ux, abs=tol)
    assert (CY * f).sum() == pytest.approx(rho * uy, abs=tol)
    assert (CX * CX * f).sum() == pytest.approx(rho * ux * ux + p, rel=tol, abs=tol)
    assert (CY * CY * f).sum() == pytest.approx(rho * uy * uy + p, rel=tol, abs=tol)
    assert (CX * CY * f).sum() == pytest.approx(rho * ux * uy, abs=tol)
    c = CS2 * (th - 1.0)
    # a^eq_{xxy}: rho ux^2 uy + rho c_s^2 (theta-1) (uy delta_xx + ...) -> one delta term
    assert (HXXY * f).sum() == pytest.approx(rho * ux * ux * uy + rho * c * uy, abs=tol)
    assert (HXYY * f).sum() == pytest.approx(rho * ux * uy * uy + rho * c * ux, abs=tol)
    # a^eq_{xxyy}: u^4 part, delta-delta part (one pairing survives), u u delta part
    expect = rho * ux * ux * uy * uy + rho * CS2 ** 2 * (th - 1) ** 2 + rho * c * (ux * ux + uy * uy)
    assert (HXXYY * f).sum() == pytest.approx(expect, abs=tol)


@pytest.mark.parametrize("rho,ux,uy,th", STATES[:4])
def test_closure_relation(rho, ux, uy, th):
    """c^3 = c on D2Q9, so H_xxx vanishes on every population and the third
    diagonal equilibrium moment is lost (Sec. 2.3, closure relation)."""
    assert np.abs(HXXX).max() == 0.0
    f = oracle.feq(rho, ux, uy, th)
    assert abs((HXXX * f).sum()) < 1e-15


def test_third_order_truncation_drops_xxyy():
    """The original model stops at third order (Sec. 2.3): its xxyy moment is
    the lattice-aliased value, the others are unchanged."""
    rho, ux, uy, th = STATES[0]
    f4 = oracle.feq(rho, ux, uy, th, order=4)
    f3 = oracle.feq(rho, ux, uy, th, order=3)
    for H in (np.ones(9), CX, CY, HXX, HXY, HYY, HXXY, HXYY):
        assert (H * f4).sum() == pytest.approx((H * f3).sum(), abs=1e-14)
    assert abs((HXXYY * f4).sum() - (HXXYY * f3).sum()) > 1e-6


@pytest.mark.parametrize("Exx,Eyy", [(0.3, -0.7), (1e-3, 2e-3), (-0.5, 0.0)])
def test_psi_moments(Exx, Eyy):
    """psi has no mass or momentum and its second Hermite moment is E
    (Sec. 2.3: 'E is the second-order Hermite moment of psi')."""
    ps = oracle.psi(Exx, Eyy)
    assert abs(ps.sum()) < 1e-15
    assert abs((CX * ps).sum()) < 1e-15 and abs((CY * ps).sum()) < 1e-15
    assert (HXX * ps).sum() == pytest.approx(Exx, abs=1e-15)
    assert (HYY * ps).sum() == pytest.approx(Eyy, abs=1e-15)
    assert abs((HXY * ps).sum()) < 1e-15


def test_f1_projection_recovers_coefficients():
    """The regularised off-equilibrium population carries exactly the six
    supplied Hermite coefficients (xx, xy, yy, xxy, yyx, xxyy) and no mass or
    momentum (Sec. 3.3)."""
    for _ in range(5):
        a = rng.normal(size=6)
        f = oracle.f1_raw(a)
        assert abs(f.sum()) < 1e-14
        assert abs((CX * f).sum()) < 1e-14 and abs((CY * f).sum()) < 1e-14
        got = [(HXX * f).sum(), (HXY * f).sum(), (HYY * f).sum(),
               (HXXY * f).sum(), (HXYY * f).sum(), (HXXYY * f).sum()]
        np.testing.assert_allclose(got, a, atol=1e-14)


def test_hermite_orthogonality():
    """Discrete orthogonality of the D2Q9 basis with the lattice weights:
    norms 2/9 (xx, yy... via H_xx H_xx), 1/9 (xy), 2/27 (xxy), 4/81 (xxyy),
    cross terms zero."""
    W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    basis = {"0": np.ones(9), "x": CX, "y": CY, "xy": HXY, "xxy": HXXY,
             "xyy": HXYY, "xxyy": HXXYY}
    # build H from the oracle's own Hermite function
    def h(i, idx):
        return oracle.hermite(i, idx)
    ora = {
        "0": np.array([h(i, []) for i in range(9)]),
        "x": np.array([h(i, [0]) for i in range(9)]),
        "y": np.array([h(i, [1]) for i in range(9)]),
        "xy": np.array([h(i, [0, 1]) for i in range(9)]),
        "xxy": np.array([h(i, [0, 0, 1]) for i in range(9)]),
        "xyy": np.array([h(i, [0, 1, 1]) for i in range(9)]),
        "xxyy": np.array([h(i, [0, 0, 1, 1]) for i in range(9)]),
    }
    for k in basis:
        np.testing.assert_allclose(ora[k], basis[k], atol=1e-15)
    # permutation symmetry of the oracle's tensors
    for i in range(9):
        assert h(i, [0, 1, 0]) == pytest.approx(h(i, [0, 0, 1]), abs=1e-15)
        assert h(i, [1, 0, 1, 0]) == pytest.approx(h(i, [0, 0, 1, 1]), abs=1e-15)
    norms = {k: (W * ora[k] * ora[k]).sum() for k in ora}
    assert norms["xy"] == pytest.approx(1 / 9)
    assert norms["xxy"] == pytest.approx(2 / 27)
    assert norms["xxyy"] == pytest.approx(4 / 81)
    keys = list(ora)
    for a in range(len(keys)):
        for b in range(a + 1, len(keys)):
            assert abs((W * ora[keys[a]] * ora[keys[b]]).sum()) < 1e-15


def test_van_albada_limiter():
    """Slope limiter phi(r) b with phi(r) = (r^2 + r)/(r^2 + 1), clipped at
    r <= 0: symmetric in its arguments, zero at extrema, exact for linear data,
    bounded by twice the smaller difference (TVD region)."""
    assert oracle.van_albada(1.0, 1.0) == pytest.approx(1.0)
    assert oracle.van_albada(2.0, 2.0) == pytest.approx(2.0)
    assert oracle.van_albada(1.0, -1.0) == 0.0
    assert oracle.van_albada(0.0, 1.0) == 0.0
    for _ in range(100):
        a, b = rng.normal(size=2)
        va, vb = oracle.van_albada(a, b), oracle.van_albada(b, a)
        assert va == pytest.approx(vb, rel=1e-14, abs=1e-300)
        if a * b > 0:
            assert abs(va) <= 2 * min(abs(a), abs(b)) + 1e-15
            assert np.sign(va) == np.sign(a)


def test_entropy_closure_roundtrip():
    """theta recovered from s = c_v ln(theta / rho^(gamma-1)) (Eq. Entropie
    expression) through the oracle's state equals the input theta."""
    import hlbm_inputs as hi
    r, u, v, t = hi.random_smooth(8, 6, seed=3)
    S = oracle.OracleSolver(oracle.OracleParams(8, 6, gamma=1.3), r, u, v, theta=t)
    m = S.moments()
    np.testing.assert_allclose(m["theta"], t, rtol=1e-13)
    np.testing.assert_allclose(m["rho"], r, rtol=1e-13)
    np.testing.assert_allclose(m["ux"], u, atol=1e-14)
    np.testing.assert_allclose(m["uy"], v, atol=1e-14)


def test_f1_recursion_is_galilean_shift():
    """The recursion of Sec. 3.3 is the binomial (Galilean) shift of a purely
    second-order off-equilibrium moment from the fluid frame to the lab
    frame, plus the thermal trace part: the lab-frame xxy, yyx and xxyy
    Hermite moments of f^1 are u_y a_xx + 2 u_x a_xy, u_x a_yy + 2 u_y a_xy
    and u_y^2 a_xx + u_x^2 a_yy + 4 u_x u_y a_xy + c_s^2 (theta - 1) tr a."""
    for _ in range(8):
        axx, axy, ayy = rng.normal(size=3) * 1e-2
        ux, uy = rng.uniform(-0.5, 0.5, size=2)
        th = rng.uniform(0.1, 1.2)
        f = oracle.f1(axx, axy, ayy, ux, uy, th)
        np.testing.assert_allclose((HXX * f).sum(), axx, atol=1e-15)
        np.testing.assert_allclose((HXY * f).sum(), axy, atol=1e-15)
        np.testing.assert_allclose((HYY * f).sum(), ayy, atol=1e-15)
        np.testing.assert_allclose((HXXY * f).sum(), uy * axx + 2 * ux * axy, atol=1e-15)
        np.testing.assert_allclose((HXYY * f).sum(), ux * ayy + 2 * uy * axy, atol=1e-15)
        shift = uy * uy * axx + ux * ux * ayy + 4 * ux * uy * axy
        thermal = CS2 * (th - 1.0) * (axx + ayy)
        np.testing.assert_allclose((HXXYY * f).sum(), shift + thermal, atol=1e-15)
