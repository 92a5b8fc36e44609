"""Pins of the oracle's full step against invariants and symmetries the
method must satisfy (collision invariants, Sec. 3.1; fixed points; lattice
symmetry; consistent initialisation, Sec. 3.5)."""
import numpy as np
import pytest

import hlbm_inputs as hi
import oracle


def make(nx, ny, fields, **kw):
    r, u, v, t = fields
    return oracle.OracleSolver(oracle.OracleParams(nx, ny, **kw), r, u, v, theta=t)


def test_mass_momentum_conserved_periodic():
    """rho and rho u are collision invariants and streaming permutes
    populations, so totals are constant on a periodic grid (Sec. 3.1)."""
    S = make(24, 20, hi.random_smooth(24, 20, seed=7, amp=0.05), mu=2e-3, sigma=0.5)
    t0 = S.totals()
    S.step(40)
    t1 = S.totals()
    assert abs(t1[0] - t0[0]) / t0[0] < 1e-13
    assert abs(t1[1] - t0[1]) / t0[0] < 1e-13
    assert abs(t1[2] - t0[2]) / t0[0] < 1e-13


@pytest.mark.parametrize("bc", ["periodic", "extrapolate"])
@pytest.mark.parametrize("vel", [(0.0, 0.0), (0.35, -0.2), (0.5, 0.45)])
def test_uniform_state_is_fixed_point(bc, vel):
    """A uniform (rho, u, theta) -- supersonic included -- has zero gradients,
    zero correction term and F = f^eq, so it does not change (Sec. 3.2-3.3)."""
    fields = hi.uniform(9, 7, 1.3, vel[0], vel[1], 0.2)
    S = make(9, 7, fields, bc_x=bc, bc_y=bc, mu=1e-2, sigma=0.7)
    m0 = S.moments()
    S.step(15)
    m1 = S.moments()
    for k in ("rho", "ux", "uy", "theta"):
        np.testing.assert_allclose(m1[k], m0[k], rtol=1e-14, atol=1e-15)


def test_zero_viscosity_uniform_entropy_stays_uniform():
    """With mu = 0 (so lambda = 0 and Phi = 0) a uniform s has zero MUSCL
    slopes and differences, so it is carried bitwise unchanged even though the
    flow is not uniform (Eq. sequaalgo)."""
    nx, ny = 20, 16
    r, u, v, t = hi.random_smooth(nx, ny, seed=5, amp=0.02)
    s = np.full((ny, nx), -1.234)
    S = oracle.OracleSolver(oracle.OracleParams(nx, ny, mu=0.0), r, u, v, s=s)
    S.step(10)
    assert np.array_equal(S.moments()["s"], s)


def test_sigma0_phi_lbm_equals_fd():
    """For sigma = 0 the LBM form of the viscous heat, -(tau/taubar) a1 : grad u
    with a1 = a1FD, equals the finite-difference form mu S : grad u
    (Eq. viscous heat discret)."""
    nx, ny = 16, 14
    f = hi.random_smooth(nx, ny, seed=11, amp=0.05)
    A = make(nx, ny, f, mu=5e-3, sigma=0.0, phi_mode="lbm")
    B = make(nx, ny, f, mu=5e-3, sigma=0.0, phi_mode="fd")
    A.step(1)
    B.step(1)
    pa, pb = A.field("phi"), B.field("phi")
    assert np.abs(pb).max() > 0
    np.testing.assert_allclose(pa, pb, rtol=1e-12, atol=1e-14 * np.abs(pb).max())
    assert (pb >= -1e-18).all()  # FD form is a sum of squares
    A.step(10)
    B.step(10)
    for k in ("rho", "ux", "uy", "s"):
        np.testing.assert_allclose(A.moments()[k], B.moments()[k], rtol=1e-12, atol=1e-14)


def test_sigma_positive_phi_differs():
    """With sigma > 0 the LBM form uses the projected a1 and differs from FD."""
    nx, ny = 16, 14
    f = hi.random_smooth(nx, ny, seed=11, amp=0.05)
    A = make(nx, ny, f, mu=5e-3, sigma=0.9, phi_mode="lbm")
    B = make(nx, ny, f, mu=5e-3, sigma=0.9, phi_mode="fd")
    A.step(3)
    B.step(3)
    assert np.abs(A.field("phi") - B.field("phi")).max() > 1e-9


def test_initialisation_natural_off_equilibrium():
    """Initialisation builds F^0 = f^eq + f1[a1FD] - psi/2, so the projected
    a1PR of F^0 equals a1FD (Algorithm step 3) and moments return (rho, u)."""
    nx, ny = 12, 10
    f = hi.random_smooth(nx, ny, seed=2, amp=0.05)
    A = make(nx, ny, f, mu=4e-3, sigma=1.0)   # a1 = a1PR
    B = make(nx, ny, f, mu=4e-3, sigma=0.0)   # a1 = a1FD
    for k in ("a1xx", "a1xy", "a1yy"):
        a, b = A.field(k), B.field(k)
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-15)
    # traceless FD stress (Eq. a1FD with D = 2)
    np.testing.assert_allclose(B.field("a1xx") + B.field("a1yy"), 0.0, atol=1e-17)


def _transpose_fields(f):
    r, u, v, t = f
    return r.T.copy(), v.T.copy(), u.T.copy(), t.T.copy()


@pytest.mark.parametrize("bcs", [("periodic", "periodic"), ("extrapolate", "periodic")])
def test_transpose_symmetry(bcs):
    """Swapping x and y (and u_x, u_y) commutes with the step: the D2Q9
    lattice and every stencil are symmetric under the diagonal reflection."""
    nx, ny = 18, 14
    f = hi.random_smooth(nx, ny, seed=21, amp=0.04)
    A = make(nx, ny, f, mu=3e-3, sigma=0.4, bc_x=bcs[0], bc_y=bcs[1])
    B = make(ny, nx, _transpose_fields(f), mu=3e-3, sigma=0.4, bc_x=bcs[1], bc_y=bcs[0])
    A.step(12)
    B.step(12)
    ma, mb = A.moments(), B.moments()
    np.testing.assert_allclose(mb["rho"], ma["rho"].T, rtol=1e-13)
    np.testing.assert_allclose(mb["ux"], ma["uy"].T, atol=1e-14)
    np.testing.assert_allclose(mb["uy"], ma["ux"].T, atol=1e-14)
    np.testing.assert_allclose(mb["s"], ma["s"].T, rtol=1e-13, atol=1e-14)


def test_mirror_symmetry():
    """Reflecting x -> -x (and u_x -> -u_x) commutes with the step; this
    catches a wrong upwind direction or lattice velocity sign."""
    nx, ny = 17, 12
    r, u, v, t = hi.random_smooth(nx, ny, seed=8, amp=0.05, u0=(0.3, 0.1))
    A = make(nx, ny, (r, u, v, t), mu=2e-3, sigma=0.3)
    B = make(nx, ny, (r[:, ::-1].copy(), -u[:, ::-1].copy(), v[:, ::-1].copy(),
                      t[:, ::-1].copy()), mu=2e-3, sigma=0.3)
    A.step(12)
    B.step(12)
    ma, mb = A.moments(), B.moments()
    np.testing.assert_allclose(mb["rho"], ma["rho"][:, ::-1], rtol=1e-13)
    np.testing.assert_allclose(mb["ux"], -ma["ux"][:, ::-1], atol=1e-14)
    np.testing.assert_allclose(mb["uy"], ma["uy"][:, ::-1], atol=1e-14)
    np.testing.assert_allclose(mb["s"], ma["s"][:, ::-1], rtol=1e-13, atol=1e-14)


def test_checkpoint_resume_bitwise():
    """The state (F, s) is the whole state: saving after N steps and resuming
    gives bitwise the same result as running 2N steps."""
    nx, ny = 14, 11
    f = hi.random_smooth(nx, ny, seed=4, amp=0.04)
    A = make(nx, ny, f, mu=3e-3, sigma=0.5)
    A.step(8)
    F, s = A.state()
    B = make(nx, ny, f, mu=3e-3, sigma=0.5)
    B.set_state(F, s)
    A.step(8)
    B.step(8)
    FA, sA = A.state()
    FB, sB = B.state()
    assert np.array_equal(FA, FB) and np.array_equal(sA, sB)


def test_translation_equivariance_periodic():
    """Shifting the periodic initial field shifts the result identically."""
    nx, ny = 15, 13
    r, u, v, t = hi.random_smooth(nx, ny, seed=9, amp=0.04)
    sh = (3, 5)
    A = make(nx, ny, (r, u, v, t), mu=3e-3, sigma=0.5)
    B = make(nx, ny, tuple(np.roll(a, sh, axis=(0, 1)) for a in (r, u, v, t)), mu=3e-3, sigma=0.5)
    A.step(6)
    B.step(6)
    for k in ("rho", "ux", "uy", "s"):
        np.testing.assert_array_equal(B.moments()[k], np.roll(A.moments()[k], sh, axis=(0, 1)))


def test_extrapolation_boundary_zero_gradient_inflow():
    """Zero-gradient boundaries: a uniform supersonic stream entering at the
    left boundary stays uniform (ghost state = copy of the boundary node)."""
    fields = hi.uniform(30, 3, 1.0, 0.45, 0.0, 0.1)
    S = make(30, 3, fields, bc_x="extrapolate", mu=1e-3)
    S.step(50)
    m = S.moments()
    np.testing.assert_allclose(m["ux"], 0.45, rtol=1e-13)
