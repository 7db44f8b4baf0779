"""Planted mistakes in the oracle's plant equations, each caught by a pin other than the
integrator-vs-matrix-exponential one.

Every case copies the oracle's C source with ONE coefficient of the model (Section 2.1 components,
Table 1 parameters) changed, builds it with gcc on the CPU and evaluates the equation-level pins on
it: the regression anchor (theta samples, peak velocity, eigenvalues of both pieces), the fixation
statics (steady state = amplitude, force balance for arbitrary levels, the closed-form equilibrium
zeroing every derivative) and rest at the pulse onset.
The closed-form test probes A from the oracle's own right-hand side, so it would pass with a wrong
equation; these pins do not depend on the oracle being right.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from test_oracle import anchor_eigen_errors, anchor_trajectory_errors

SRC = os.path.join(os.path.dirname(oracle.__file__), "opmm_oracle.c")

# (name, original text, mutated text): one coefficient of one equation each
MUTATIONS = [
    ("globe: antagonist series tension dropped", "dx[1] = (t_se_ag - t_se_ant - q.bp * w", "dx[1] = (t_se_ag - q.bp * w"),
    ("globe: passive viscosity x1.1", "- q.bp * w -", "- 1.1 * q.bp * w -"),
    ("globe: passive elasticity x1.1", "- q.kp * th) / q.j", "- 1.1 * q.kp * th) / q.j"),
    ("globe: inertia x1.1", "- q.kp * th) / q.j", "- q.kp * th) / (1.1 * q.j)"),
    ("passive elasticity without N_C_AG", "q->kp = p[7] + p[8];", "q->kp = p[8];"),
    ("agonist series elasticity x1.1", "double t_se_ag = q.kse_ag * (xa - th);", "double t_se_ag = 1.1 * q.kse_ag * (xa - th);"),
    ("antagonist series element sign", "double t_se_ant = q.kse_ant * (xn + th);", "double t_se_ant = q.kse_ant * (xn - th);"),
    ("agonist length-tension x1.1", "dx[2] = (fa - q.klt_ag * xa", "dx[2] = (fa - 1.1 * q.klt_ag * xa"),
    ("antagonist length-tension x1.1", "dx[3] = (fn - q.klt_ant * xn", "dx[3] = (fn - 1.1 * q.klt_ant * xn"),
    ("agonist force-velocity x1.1", "- t_se_ag) / q.b_ag;", "- t_se_ag) / (1.1 * q.b_ag);"),
    ("antagonist force-velocity x1.1", "- t_se_ant) / q.b_ant;", "- t_se_ant) / (1.1 * q.b_ant);"),
    ("agonist active-state time constant x1.1", "dx[4] = (n_ag - fa) / tau_ag;", "dx[4] = (n_ag - fa) / (1.1 * tau_ag);"),
    ("antagonist active-state time constant x1.1", "dx[5] = (n_ant - fn) / tau_ant;", "dx[5] = (n_ant - fn) / (1.1 * tau_ant);"),
    ("muscles swapped in the active states", "dx[4] = (n_ag - fa) / tau_ag;", "dx[4] = (n_ag - fa) / tau_ant;"),
    ("activation time constants in the wrong unit", "q->tac_ag = p[10] * 1e-3;", "q->tac_ag = p[10] * 1.1e-3;"),
    ("deactivation time constant of the agonist x1.1", "q->tde_ag = p[12] * 1e-3;", "q->tde_ag = p[12] * 1.1e-3;"),
    ("pulse width x1.05", "q->pw = p[17] * 1e-3;", "q->pw = p[17] * 1.05e-3;"),
    ("agonist tension slope x1.1 in the step", "double t_ag = p[14] + p[7] * th;", "double t_ag = p[14] + 1.1 * p[7] * th;"),
    ("antagonist tension slope sign in the step", "double t_ant = p[14] - p[8] * th;", "double t_ant = p[14] + p[8] * th;"),
    ("agonist step without the length-tension term", "*s_ag = t_ag * (p[0] + p[2]) / p[0] + p[2] * th;", "*s_ag = t_ag * (p[0] + p[2]) / p[0];"),
    ("antagonist step share inverted", "*s_ant = t_ant * (p[1] + p[3]) / p[1] - p[3] * th;", "*s_ant = t_ant * (p[1] + p[3]) / p[3] - p[3] * th;"),
    ("equilibrium share c_ag inverted", "double c_ag = q.kse_ag / (q.kse_ag + q.klt_ag);", "double c_ag = q.klt_ag / (q.kse_ag + q.klt_ag);"),
    ("equilibrium without passive elasticity", "/ (q.kp + c_ag * q.klt_ag + c_ant * q.klt_ant);", "/ (c_ag * q.klt_ag + c_ant * q.klt_ant);"),
    ("pulse height of the antagonist from the agonist", "lv[3] = p[16];", "lv[3] = p[15];"),
]


def _build(tmp_path, i, src):
    c = tmp_path / ("mut%02d.c" % i)
    so = tmp_path / ("libmut%02d.so" % i)
    c.write_text(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-ffp-contract=off", "-shared", "-fPIC", "-o", str(so), str(c),
                           "-lm", "-lpthread"])
    L = ctypes.CDLL(str(so))
    P, d, i_ = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    L.oracle_rhs.argtypes = [P, P, d, d, d, d, P]
    L.oracle_simulate.argtypes = [P, d, i_, d, i_, P]
    L.oracle_simulate.restype = i_
    L.oracle_simulate_levels.argtypes = [P, P, i_, d, i_, P, P]
    L.oracle_simulate_levels.restype = i_
    L.oracle_control_levels.argtypes = [P, d, P]
    L.oracle_equilibrium.argtypes = [P, d, d, P]
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pins_failed(L):
    """Names of the equation-level pins the library fails."""
    def simulate(p, amp, T, dt, nsub=8):
        p = np.ascontiguousarray(p, np.float64); th = np.zeros(T)
        assert L.oracle_simulate(_ptr(p), float(amp), int(T), float(dt), nsub, _ptr(th)) == 0
        return th

    def rhs(p, x, n_ag, n_ant, ta, tn):
        p = np.ascontiguousarray(p, np.float64); x = np.ascontiguousarray(x, np.float64); dx = np.zeros(6)
        L.oracle_rhs(_ptr(p), _ptr(x), float(n_ag), float(n_ant), float(ta), float(tn), _ptr(dx))
        return dx

    failed = []
    err, verr = anchor_trajectory_errors(simulate)
    if not (err <= 5e-4 + 1e-12 and verr < 1.0):
        failed.append("anchor trajectory")
    if not anchor_eigen_errors(rhs) < 1e-3:
        failed.append("anchor eigenvalues")
    rng = np.random.default_rng(11)
    for _ in range(3):
        amp = rng.uniform(2, 30)
        p = oracle.nominal(2.2 * amp + 21) * rng.uniform(0.7, 1.3, 18)
        th = simulate(p, amp, 3000, 1.0, nsub=4)
        if not (abs(th[-1] - amp) < 1e-8 and abs(th[0]) < 1e-12):
            failed.append("steady state / rest")
            break
    p = oracle.nominal(43.0) * rng.uniform(0.7, 1.3, 18)
    lv = np.zeros(6)
    L.oracle_control_levels(_ptr(np.ascontiguousarray(p)), 0.0, _ptr(lv))
    lv[2:] = [40.0, 3.0, 31.0, 12.0]
    th = np.zeros(3000)
    L.oracle_simulate_levels(_ptr(np.ascontiguousarray(p)), _ptr(lv), 3000, 1.0, 4, _ptr(th), None)
    ca = p[0] / (p[0] + p[2]); cn = p[1] / (p[1] + p[3])
    ss = (ca * lv[4] - cn * lv[5]) / (p[7] + p[8] + ca * p[2] + cn * p[3])
    if not abs(th[-1] - ss) < 1e-8:
        failed.append("force balance")
    xe = np.zeros(6)
    L.oracle_equilibrium(_ptr(np.ascontiguousarray(p)), 31.0, 12.0, _ptr(xe))
    de = rhs(p, xe, 31.0, 12.0, 1e-3, 1e-3)
    if not np.abs(de).max() < 1e-9 * max(1.0, np.abs(xe).max() / p[9]):
        failed.append("equilibrium at arbitrary active states")
    return failed


def test_unmutated_source_passes(tmp_path):
    assert _pins_failed(_build(tmp_path, 99, open(SRC).read())) == []


@pytest.mark.parametrize("i", range(len(MUTATIONS)), ids=[m[0] for m in MUTATIONS])
def test_planted_equation_mistake_is_caught(tmp_path, i):
    name, old, new = MUTATIONS[i]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation target not unique: " + name
    failed = _pins_failed(_build(tmp_path, i, src.replace(old, new)))
    assert failed, "no equation-level pin catches: " + name
