"""Closed-form pins of the oracle's pointwise fluxes and of the compact-DG
face lifting.

The viscous flux follows the Navier-Stokes equations of Sec. 4 (eqs.
ns1-ns5): Newtonian stress with Stokes' hypothesis, Fourier heat conduction
through the Prandtl number, and the viscous work u . tau in the energy
equation.  Each test below fixes the state and its *primitive* gradients
(density, velocity, specific internal energy), builds the conservative
gradients the oracle takes, and compares with what continuum mechanics gives
for that flow: zero stress under rigid rotation, the shear stress of a
uniform shear, the normal stresses of a pure dilatation, Fourier's law at
rest, and frame invariance.  The numerical flux is pinned by consistency,
conservation, rotational invariance and the pure-pressure flux through a
face moving with the fluid.  The lifting of the compact DG treatment (the
reading of the viscous discretisation the paper delegates, Sec. 4.1) is
pinned by its defining identity against closed-form edge and element
integrals.
"""
import math

import numpy as np
import pytest

GAMMA, PR, RE, MACH = 1.4, 0.72, 1000.0, 0.2
MU_V = 1.0 / RE


def make(O, **kw):
    base = dict(Nr=2, Nth=6, p=1, Nt=4)
    base.update(kw)
    return O.Oracle(**base)


def conservative(rho, u, e, grho, gu, ge):
    """State U = (rho, rho u, rho E) and its gradient dU[m][d] from the
    primitive state and primitive gradients (E = e + |u|^2 / 2)."""
    u = np.asarray(u, float)
    gu = np.asarray(gu, float)          # gu[i][d] = d u_i / d x_d
    grho = np.asarray(grho, float)
    ge = np.asarray(ge, float)
    E = e + 0.5 * u @ u
    gE = ge + u @ gu                    # d/dx_d (e + |u|^2/2)
    U = np.array([rho, rho * u[0], rho * u[1], rho * E])
    dU = np.zeros((4, 2))
    dU[0] = grho
    dU[1] = u[0] * grho + rho * gu[0]
    dU[2] = u[1] * grho + rho * gu[1]
    dU[3] = E * grho + rho * gE
    return U, dU


STATE = dict(rho=1.3, u=(0.4, -0.2), e=30.0, grho=(0.7, -1.1))


def test_rigid_rotation_has_no_viscous_stress(oracle_mod):
    """A rigid rotation u = omega x (-y, x) has no strain: tau = 0, so with a
    uniform temperature every viscous flux vanishes, whatever the density
    gradient."""
    o = make(oracle_mod)
    w = 2.5
    U, dU = conservative(gu=[[0.0, -w], [w, 0.0]], ge=(0.0, 0.0), **STATE)
    F = o.flux_vis(U, dU)
    assert np.abs(F).max() <= 1e-15 * 50


def test_uniform_shear_stress(oracle_mod):
    """u_x = a y: tau_xy = tau_yx = mu a, normal stresses zero; the energy
    flux is the viscous work u_i tau_id."""
    o = make(oracle_mod)
    a = 3.0
    U, dU = conservative(gu=[[0.0, a], [0.0, 0.0]], ge=(0.0, 0.0), **STATE)
    F = o.flux_vis(U, dU)
    u = np.array(STATE["u"])
    tau = MU_V * np.array([[0.0, a], [a, 0.0]])
    assert np.allclose(F[0], 0.0, atol=1e-15)
    assert np.allclose(F[1:3], tau, rtol=1e-13, atol=1e-16)
    assert np.allclose(F[3], u @ tau, rtol=1e-13, atol=1e-16)


def test_uniform_dilatation_stokes_hypothesis(oracle_mod):
    """u = a x (pure expansion, div u = 2a): with the bulk viscosity -2 mu / 3
    of the stress tensor of Sec. 4 the normal stresses are
    mu (2a - 2/3 * 2a) = 2 mu a / 3 and the shear stress is zero."""
    o = make(oracle_mod)
    a = -1.7
    U, dU = conservative(gu=[[a, 0.0], [0.0, a]], ge=(0.0, 0.0), **STATE)
    F = o.flux_vis(U, dU)
    assert np.allclose(F[1:3], (2.0 / 3.0) * MU_V * a * np.eye(2), rtol=1e-13, atol=1e-17)


def test_fourier_heat_conduction_at_rest(oracle_mod):
    """Fluid at rest with a temperature gradient: the only viscous flux is the
    conductive energy flux k grad T with k = mu c_p / Pr.  For a calorically
    perfect gas c_p T = gamma e, so the energy flux is (mu / Pr) gamma grad e;
    the adiabatic variant (heat = 0) has none.  The density gradient (and so
    the pressure gradient) must not contribute."""
    o = make(oracle_mod)
    ge = np.array([0.9, -2.3])
    U, dU = conservative(rho=1.3, u=(0.0, 0.0), e=30.0, grho=(0.7, -1.1), gu=np.zeros((2, 2)), ge=ge)
    F = o.flux_vis(U, dU)
    assert np.allclose(F[:3], 0.0, atol=1e-16)
    assert np.allclose(F[3], MU_V / PR * GAMMA * ge, rtol=1e-13)
    F0 = o.flux_vis(U, dU, heat=False)
    assert np.allclose(F0, 0.0, atol=1e-16)


def rot(th):
    return np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])


def rotate_state(Q, U):
    return np.array([U[0], *(Q @ U[1:3]), U[3]])


def test_viscous_flux_is_frame_invariant(oracle_mod):
    """Rotating the frame by Q: the state's momentum and every gradient rotate,
    and the flux transforms as F' = Q_m F Q^T (Q_m acting on the momentum
    rows): the stress is a tensor, the heat flux and the viscous work are
    vectors."""
    o = make(oracle_mod)
    g = np.random.Generator(np.random.PCG64(11))
    U, dU = conservative(rho=1.1, u=(0.3, 0.5), e=25.0, grho=g.standard_normal(2), gu=g.standard_normal((2, 2)),
                         ge=g.standard_normal(2))
    Q = rot(0.83)
    Qm = np.eye(4)
    Qm[1:3, 1:3] = Q
    U2 = Qm @ U
    dU2 = Qm @ dU @ Q.T
    F = o.flux_vis(U, dU)
    F2 = o.flux_vis(U2, dU2)
    assert np.allclose(F2, Qm @ F @ Q.T, rtol=1e-12, atol=1e-14)


def euler_state(rho, u, p):
    u = np.asarray(u, float)
    return np.array([rho, rho * u[0], rho * u[1], p / (GAMMA - 1) + 0.5 * rho * u @ u])


def test_flux_through_a_face_moving_with_the_fluid_is_pressure_only(oracle_mod):
    """When the face moves with the normal velocity of the fluid
    (u . n = v_G . n) nothing crosses it: the mass flux is zero, the momentum
    flux is p n and the energy flux is the pressure work p (v_G . n)."""
    o = make(oracle_mod)
    n = np.array([0.6, 0.8])
    u = np.array([0.35, -0.15])
    p = 17.0
    U = euler_state(1.2, u, p)
    vn = u @ n
    H = o.flux_h(U, n, vn)
    assert abs(H[0]) <= 1e-15
    assert np.allclose(H[1:3], p * n, rtol=1e-14)
    assert abs(H[3] - p * vn) <= 1e-13 * p


def test_numerical_flux_consistency_conservation_invariance(oracle_mod):
    """Fhat(U, U) = H(U) (consistency); Fhat(UL, UR; n, vn) = -Fhat(UR, UL;
    -n, -vn) (the flux leaving one side enters the other); and rotating the
    frame rotates the momentum flux."""
    o = make(oracle_mod)
    UL = euler_state(1.1, (0.5, 0.1), 16.0)
    UR = euler_state(0.9, (0.2, -0.3), 19.0)
    n = np.array([math.cos(1.1), math.sin(1.1)])
    vn = 0.27
    assert np.allclose(o.flux_lf(UL, UL, n, vn), o.flux_h(UL, n, vn), rtol=1e-15, atol=1e-14)
    assert np.allclose(o.flux_lf(UL, UR, n, vn), -o.flux_lf(UR, UL, -n, -vn), rtol=1e-14, atol=1e-13)
    Q = rot(-0.6)
    F = o.flux_lf(UL, UR, n, vn)
    F2 = o.flux_lf(rotate_state(Q, UL), rotate_state(Q, UR), Q @ n, vn)
    assert np.allclose(F2, rotate_state(Q, F), rtol=1e-13, atol=1e-13)
    # the flux of a jump is dissipative: it differs from the central average
    # by -alpha (UR - UL) / 2 with alpha > 0 of the order of the sound speed
    avg = 0.5 * (o.flux_h(UL, n, vn) + o.flux_h(UR, n, vn))
    alpha = -2.0 * (F - avg) / (UR - UL)
    assert np.allclose(alpha, alpha[0], rtol=1e-12) and 3.0 < alpha[0] < 6.0


# ---------------------------------------------------------------- lifting
# Newton-Cotes weights of the equispaced Lagrange basis: int_T phi_a = |T| w_a
# (p = 1: 1/3 each; p = 2: 0 at the vertices, 1/3 at the edge nodes; p = 3:
# 1/30 at the vertices, 3/40 at the edge nodes, 9/20 at the centroid)
def nc_weights(p):
    nodes = [(s, t) for t in range(p + 1) for s in range(p + 1 - t)]
    w = []
    for s, t in nodes:
        r = p - s - t
        nvert = [s, t, r].count(p)
        nzero = [s, t, r].count(0)
        if p == 1:
            w.append(1 / 3)
        elif p == 2:
            w.append(0.0 if nvert else 1 / 3)
        else:
            w.append(1 / 30 if nvert else (3 / 40 if nzero else 9 / 20))
    return np.array(w)


def edge_of(ev, vxy, K, f):
    """length and outward unit normal of local face f (vertex f -> f+1) of K
    (counter-clockwise triangles: the outward normal is the edge direction
    turned clockwise)"""
    a = vxy[ev[K, f]]
    b = vxy[ev[K, (f + 1) % 3]]
    t = b - a
    L = float(np.hypot(*t))
    return L, np.array([t[1], -t[0]]) / L


def interior_faces(en):
    return [(K, f) for K in range(en.shape[0]) for f in range(3) if en[K, f] >= 0]


@pytest.mark.parametrize("p", [1, 3])
def test_lifting_of_a_constant_jump(oracle_mod, p):
    """With the mesh at rest and U^L - U^R = c along the face, testing the
    lifting's definition with the constant tau = e_m e_D gives
    int_L r_e = -|e| c_m N^L_D.  The lifting lives on the lower-index side,
    and moving the jump to the other side flips its sign."""
    o = make(oracle_mod, p=p)
    o.set_params(np.zeros(3))
    ev, en, tw, vxy = o.mesh()
    _, area = o.nodes()
    w = nc_weights(p)
    c = np.array([0.01, -0.02, 0.03, 0.5])
    # every local face index on both kinds of triangle, inner and outer ring
    faces = interior_faces(en)
    for K, f in faces[::max(1, len(faces) // 12)]:
        nb = int(en[K, f])
        assert nb >= 0
        L = min(K, nb)
        fL = f if L == K else int(tw[K, f])
        length, N = edge_of(ev, vxy, L, fL)
        for side, sign in ((L, 1.0), (max(K, nb), -1.0)):
            u = o.freestream()
            u.reshape(o.Ne, o.np, 4)[side] += c
            lift, on_K = o.face_lift(0, 0, u, K, f)
            assert on_K == (K == L)
            integral = area[L] * np.einsum("a,amd->md", w, lift)
            assert np.allclose(integral, -sign * length * np.outer(c, N), rtol=1e-12, atol=1e-15), (K, f, side)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_lifting_vanishes_for_a_continuous_field(oracle_mod, p):
    """A field continuous across every face (the nodal values of one global
    linear function on every element) has no jumps, hence no lifting."""
    o = make(oracle_mod, p=p)
    o.set_params(np.zeros(3))
    ev, en, tw, vxy = o.mesh()
    X, _ = o.nodes()
    u = o.freestream().reshape(o.Ne, o.np, 4)
    u += 0.01 * X[..., 0:1] * np.array([1.0, 2.0, -1.0, 3.0]) - 0.02 * X[..., 1:2] * np.array([0.5, 1.0, 1.0, 2.0])
    for K, f in interior_faces(en):
        lift, _ = o.face_lift(0, 0, u.ravel(), K, f)
        assert np.abs(lift).max() <= 1e-12, (K, f)


def test_lifting_of_a_linear_jump_p1(oracle_mod):
    """p = 1 and a jump linear along the edge: the lifting solves
    M r_m,D = -N_D int_e phi [U_m] ds with the closed-form P1 mass matrix
    |L|/12 [[2,1,1],[1,2,1],[1,1,2]], and the edge integral of a product of
    two linear functions by Simpson's rule (exact for quadratics)."""
    o = make(oracle_mod, p=1)
    o.set_params(np.zeros(3))
    ev, en, tw, vxy = o.mesh()
    _, area = o.nodes()
    K, f = 5, 1
    nb = int(en[K, f])
    L = min(K, nb)
    fL = f if L == K else int(tw[K, f])
    length, N = edge_of(ev, vxy, L, fL)
    g = np.random.Generator(np.random.PCG64(3))
    d = 0.01 * g.standard_normal((3, 4))       # added to L's three nodes: jump linear on the edge
    u = o.freestream()
    u.reshape(o.Ne, 3, 4)[L] += d
    lift, _ = o.face_lift(0, 0, u, K, f)
    # P1 nodes are the vertices in order; the edge fL joins nodes fL, fL+1
    a, b = fL, (fL + 1) % 3
    rhs = np.zeros((3, 4))
    # Simpson on [0, 1]: int phi_i [U] ds over the edge, phi_a = 1 - s, phi_b = s
    for s, ws in ((0.0, 1 / 6), (0.5, 4 / 6), (1.0, 1 / 6)):
        jump = (1 - s) * d[a] + s * d[b]
        rhs[a] += ws * (1 - s) * jump
        rhs[b] += ws * s * jump
    rhs *= length
    M = area[L] / 12.0 * np.array([[2.0, 1, 1], [1, 2, 1], [1, 1, 2]])
    expect = -np.einsum("am,d->amd", np.linalg.solve(M, rhs), N)
    assert np.allclose(lift, expect, rtol=1e-12, atol=1e-15)
