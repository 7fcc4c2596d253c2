"""The oracle's pins catch plausible mistakes.

Each case plants one slip in a copy of oracle/oracle.c, compiles the copy
into a temporary library (the committed oracle is untouched), loads it
through a separate instance of the oracle's binding, and runs the pin that
should catch the slip: that pin must then fail.  The slips are the ones a
reader checking the code against the paper could miss:
- the radial stretching and a twin-face index of the O-grid;
- the sign of the grid-velocity flux of the ALE form;
- in the primal sweep: the time step dropped from the stage equation, the
  stage sum with the tableau transposed and the state update weighted with
  the stage times (Sec. 2.1 eq. dirk), caught by the rows of eq.
  abs-govern-disc;
- the bulk viscosity coefficient of Stokes' hypothesis (Sec. 4, eqs. ns1-ns5);
- the heat flux built from (gamma - 1) instead of gamma;
- the sign and the scale of the compact-DG lifting;
- the transposed block product with untransposed blocks (caught by the
  stage systems' adjoint identity);
- a neighbour's Jacobian block stored in the wrong block slot, and the
  parameter derivatives taken in the wrong parameter (caught by central
  differences);
- a dropped stage coupling in the tangent sweep (eq. dirk-sens-mvp);
- a transposed tableau index and a missing transpose in the backward sweep
  (eq. uns-disc-adj-dirk-sens-mvp), caught by the duality theorem of the
  appendix;
- a GCL stage value that leaves out its own stage's slope (an explicit
  instead of the diagonally implicit recurrence), caught by the third-order
  pin;
- the sign of Alg. 3's right-hand side (the paper's printed residual and
  update disagree in sign), caught by the dense solve;
- the time step dropped from the gradient sum (eq. funcl-grad-nosens-dirk),
  the QoI forcing of the backward stages without its tableau factor and the
  explicit parameter term without the quadrature weights, caught by the
  direct method;
- the wall's reflected state built about a wall at rest instead of the
  moving wall (reading of the no-slip wall), caught by the QoIs' closed
  forms, whose fluid moves with the wall;
- the power built with the velocity components swapped, and the force of
  the body on the fluid in place of the fluid's on the body (Sec. 4 eq.
  qoi), caught by the QoIs' closed forms;
- the period average weighted with the stage times instead of the
  quadrature weights, caught by the solver-consistent QoI pin.
The same is done for the plain-numpy references of the learned form: the
tanh derivative of the perceptron's back-propagation, and the centring and
the mode scaling of the POD.
A control copy with no slip, built the same way, passes every one of these
pins, so a failure below is the slip's and not the harness's."""
import importlib.util
import os
import subprocess
import types

import pytest

import test_mlp_oracle as M
import test_oracle_flux_pins as F
import test_oracle_pins as P
import test_oracle_pod_pins as D
from paper_1512_00616_amd import inputs

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


def _mutant(tmp_path, old, new):
    src = open(os.path.join(ORACLE, "oracle.c")).read()
    assert src.count(old) == 1, old
    c = tmp_path / "oracle.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-Wl,-Bsymbolic",
                           "-I", ORACLE, str(c), "-o", str(so), "-lm"])
    spec = importlib.util.spec_from_file_location("oracle_mutant_" + tmp_path.name,
                                                  os.path.join(ORACLE, "oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB_PATH = str(so)
    mod.lib()
    return mod


def _about_one_period(pin):
    """a pin of the sweeps or of the periodic boundary-value problem, run
    about a one-period trajectory from the perturbed free stream instead of
    the shot orbit: the identities it checks (duality, the dense solve of
    Alg. 3, adjoint = direct gradient) hold about any trajectory"""
    def run(mod):
        o = mod.Oracle(Nr=2, Nth=6, p=1, Nt=2, lin_solver=0, newton_atol=1e-12)
        o.set_params(P.MU)
        u0 = o.freestream(inputs.perturbation(o.Nu, seed=1))
        try:
            pin((o, u0, None))
        finally:
            o.close()
    return run


PINS = {
    "mesh": P.test_mesh_connectivity_and_orientation,
    "moving-face": F.test_flux_through_a_face_moving_with_the_fluid_is_pressure_only,
    "dilatation": F.test_uniform_dilatation_stokes_hypothesis,
    "fourier": F.test_fourier_heat_conduction_at_rest,
    "lifting": lambda m: F.test_lifting_of_a_constant_jump(m, 1),
    "gcl-order": P.test_gcl_field_third_order_in_time,
    "qoi-closed-form": lambda m: P.test_qois_of_a_linear_pressure_field_in_heave(m, 1),
    "qoi-quadrature": P.test_period_qois_are_the_dirk_quadrature_of_the_stage_qois,
    "period-rows": P.test_one_period_solves_the_update_and_stage_rows,
    "stage-systems": lambda m: P.test_stage_solves_satisfy_their_systems(m, 0),
    "jacobian": lambda m: P.test_jacobian_matches_central_differences(m, 1),
    "dr-dmu": P.test_dr_dmu_and_dqoi_match_central_differences,
    "tangent": P.test_tangent_sweep_is_derivative_of_flow_map,
    "duality": _about_one_period(P.test_adjoint_sweep_is_transpose_of_tangent_sweep),
    "dense-alg3": _about_one_period(P.test_periodic_adjoint_matches_dense_solve),
    "adjoint-vs-direct": _about_one_period(P.test_adjoint_gradient_equals_tangent_gradient),
}

SLIPS = [
    ("stretching-per-mesh-instead-of-per-cell", "mesh",
     "double q = pow(c->cfg.stretch, 8.0 / Nr);", "double q = pow(c->cfg.stretch, 1.0 / Nr);"),
    ("twin-face-index", "mesh",
     "c->enb[3 * B] = A; c->etw[3 * B] = 2;", "c->enb[3 * B] = A; c->etw[3 * B] = 1;"),
    ("grid-velocity-flux-sign", "moving-face",
     "H[m] = F[m][0] * n[0] + F[m][1] * n[1] - U[m] * vn;", "H[m] = F[m][0] * n[0] + F[m][1] * n[1] + U[m] * vn;"),
    ("bulk-viscosity", "dilatation",
     "(i == j ? 2.0 / 3.0 * div : 0.0)", "(i == j ? 1.0 / 3.0 * div : 0.0)"),
    ("heat-flux-gamma-minus-one", "fourier",
     "cplx dh = c->gam * (dE[d]", "cplx dh = (c->gam - 1.0) * (dE[d]"),
    ("lifting-sign", "lifting",
     "double s = -len / (2.0 * c->area[L]);", "double s = len / (2.0 * c->area[L]);"),
    ("lifting-scale", "lifting",
     "double s = -len / (2.0 * c->area[L]);", "double s = -len / c->area[L];"),
    ("stage-equation-without-dt", "period-rows",
     "R[q] -= c->dt * r[q];", "R[q] -= r[q];"),
    ("stage-sum-with-transposed-tableau", "period-rows",
     "acc += c->A[i - 1][j - 1] * c->tk[(int64_t)(s - i + j) * Nu + q];",
     "acc += c->A[j - 1][i - 1] * c->tk[(int64_t)(s - i + j) * Nu + q];"),
    ("state-update-with-the-stage-times", "period-rows",
     "acc += c->bw[i] * c->tk[(int64_t)((n - 1) * 3 + i) * Nu + q];",
     "acc += c->cc[i] * c->tk[(int64_t)((n - 1) * 3 + i) * Nu + q];"),
    ("transposed-product-without-transposed-blocks", "stage-systems",
     "for (int i = 0; i < b; ++i) acc += B[i * b + j] * x[(int64_t)K * b + i];",
     "for (int i = 0; i < b; ++i) acc += B[j * b + i] * x[(int64_t)K * b + i];"),
    ("jacobian-neighbour-block-in-the-wrong-slot", "jacobian",
     "int slot = 1 + c->etw[3 * Kp + f];", "int slot = 1 + f;"),
    ("parameter-derivatives-shifted-by-one", "dr-dmu",
     "if (dir > 0) mu[dir - 1] += I * CSTEP;", "if (dir > 0) mu[dir % 3] += I * CSTEP;"),
    ("tangent-drops-stage-coupling", "tangent",
     "acc += c->A[i - 1][j - 1] * dk[(int64_t)(j - 1) * Nu + q];",
     "acc += 0.0 * dk[(int64_t)(j - 1) * Nu + q];"),
    ("adjoint-tableau-index-transposed", "duality",
     "acc += c->A[j - 1][i - 1] * z[(int64_t)(j - 1) * Nu + q];",
     "acc += c->A[i - 1][j - 1] * z[(int64_t)(j - 1) * Nu + q];"),
    ("adjoint-missing-transpose", "duality",
     "pao_bsr_apply(c, J, 1, kap, zi);", "pao_bsr_apply(c, J, 0, kap, zi);"),
    ("gcl-stage-value-without-its-own-slope", "gcl-order",
     "for (int j = 1; j <= i; ++j) s += c->A[i - 1][j - 1] * kg[(int64_t)(j - 1) * nn + k];",
     "for (int j = 1; j < i; ++j) s += c->A[i - 1][j - 1] * kg[(int64_t)(j - 1) * nn + k];"),
    ("alg3-right-hand-side-sign", "dense-alg3",
     "for (int64_t k = 0; k < Nu; ++k) gF[k] = -gF[k];", "for (int64_t k = 0; k < Nu; ++k) gF[k] = gF[k];"),
    ("wall-reflects-the-velocity-about-zero", "qoi-closed-form",
     "cplx bx = 2.0 * vG[0] - ux, by = 2.0 * vG[1] - uy;", "cplx bx = vG[0] - ux, by = vG[1] - uy;"),
    ("power-with-swapped-velocity-components", "qoi-closed-form",
     "f[0] += w * (Fh[j * 4 + 1] * vG[0] + Fh[j * 4 + 2] * vG[1]);",
     "f[0] += w * (Fh[j * 4 + 1] * vG[1] + Fh[j * 4 + 2] * vG[0]);"),
    ("force-of-the-body-on-the-fluid", "qoi-closed-form",
     "f[1] += w * Fh[j * 4 + 1];", "f[1] -= w * Fh[j * 4 + 1];"),
    ("period-average-with-the-stage-times", "qoi-quadrature",
     "Jq[0] += c->dt * c->bw[i - 1] * f[0] / c->cfg.T;", "Jq[0] += c->dt * c->cc[i - 1] * f[0] / c->cfg.T;"),
    ("adjoint-stage-forcing-without-the-tableau", "adjoint-vs-direct",
     "for (int j = i; j <= 3; ++j) acc += sc * c->bw[j - 1] * c->A[j - 1][i - 1] * fp[(int64_t)(j - 1) * Nu + q];",
     "for (int j = i; j <= 3; ++j) acc += sc * c->bw[j - 1] * fp[(int64_t)(j - 1) * Nu + q];"),
    ("explicit-parameter-term-without-quadrature-weights", "adjoint-vs-direct",
     "for (int k = 0; k < 3; ++k) g[k] += sc * c->bw[i - 1] * fm[3 * fq + k];",
     "for (int k = 0; k < 3; ++k) g[k] += sc * fm[3 * fq + k];"),
    ("gradient-sum-without-dt", "adjoint-vs-direct",
     "g[k] += c->dt * dot(Nu, kap, dr + (int64_t)k * Nu);", "g[k] += dot(Nu, kap, dr + (int64_t)k * Nu);"),
]


def test_control_copy_passes_every_pin(tmp_path):
    mod = _mutant(tmp_path, "double s = -len / (2.0 * c->area[L]);", "double s = -len / (2.0 * c->area[L]);")
    for pin in PINS.values():
        pin(mod)


@pytest.mark.parametrize("name,pin,old,new", SLIPS, ids=[s[0] for s in SLIPS])
def test_pin_fails_on_the_planted_slip(tmp_path, name, pin, old, new):
    mod = _mutant(tmp_path, old, new)
    # caught by the pin's assertion, or by the oracle itself refusing to go on
    # (a stage Newton that no longer converges), never by a crash
    with pytest.raises((AssertionError, mod.OracleError)):
        PINS[pin](mod)


# ---------------------------------------------------------------- the Python references
def _py_mutant(name, old, new):
    path = os.path.join(ORACLE, name + ".py")
    src = open(path).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle_%s_mutant" % name)
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    return mod


PY_SLIPS = [
    ("tanh-derivative", "mlp", "(1.0 - acts[l] ** 2)", "(1.0 - acts[l])",
     M, "mlp", M.test_deep_gradient_matches_central_differences),
    ("pod-without-centring", "pod", "D = X - mean", "D = X",
     D, "pod", D.test_pod_recovers_constructed_modes),
    ("pod-modes-scaled-by-the-eigenvalue", "pod",
     "modes = (V[:, :k].T @ D) / np.sqrt(lam[:k])[:, None]", "modes = (V[:, :k].T @ D) / lam[:k][:, None]",
     D, "pod", D.test_modes_orthonormal_and_snapshots_reconstructed),
]


@pytest.mark.parametrize("name,module,old,new,tmod,attr,pin", PY_SLIPS, ids=[s[0] for s in PY_SLIPS])
def test_reference_pin_fails_on_the_planted_slip(monkeypatch, name, module, old, new, tmod, attr, pin):
    # the perceptron and POD references (plain numpy): the slip is planted in
    # a copy of the module's source; an unmodified copy passes the same pin
    monkeypatch.setattr(tmod, attr, _py_mutant(module, old, old))
    pin()
    monkeypatch.setattr(tmod, attr, _py_mutant(module, old, new))
    with pytest.raises(AssertionError):
        pin()
