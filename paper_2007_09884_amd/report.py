"""Results in the paper's output format (Section 3.4, Fig. 4): one CSV row per saccade with the
saccade number, the optimisation error (OptErr, the mean absolute difference between the recorded
and the simulated trace), a serial re-computation of that error for validation (CPU_check) and
the 18 OPC values under the figure's column names.  Host-side formatting only."""
from __future__ import annotations

import numpy as np

COLUMNS = ["SacNo", "OptErr", "CPU_check", "SE_ag", "SE_ant", "LT_ag", "LT_ant", "PE_ag", "PE_ant", "Vis",
           "FV_ag", "FV_ant", "Inert", "Act_ag", "Act_ant", "Deact_ag", "Deact_ant", "Step", "H_ag", "H_ant", "W"]

# Table 1 index of each OPC column of the figure: series elasticity (K_SE), length-tension (K_LT),
# tension slope (N_C), passive viscosity (B_P), force-velocity (B), inertia (J), activation and
# deactivation times, tension intercept (N_C_FIX), pulse heights (N_SAC) and pulse width (PW)
TABLE1_INDEX = [0, 1, 2, 3, 7, 8, 6, 4, 5, 9, 10, 11, 12, 13, 14, 15, 16, 17]


def rows(opc, opt_err, cpu_check=None, first: int = 1) -> list[str]:
    """CSV lines (header first).  opc [S][18] in Table 1 order, opt_err [S]; cpu_check [S] or None
    (then the column is left empty).  Saccades are numbered from `first`."""
    opc = np.asarray(opc, np.float64).reshape(-1, 18)
    err = np.asarray(opt_err, np.float64).reshape(-1)
    if err.shape[0] != opc.shape[0]:
        raise ValueError("opt_err needs one value per saccade")
    chk = None if cpu_check is None else np.asarray(cpu_check, np.float64).reshape(-1)
    if chk is not None and chk.shape[0] != opc.shape[0]:
        raise ValueError("cpu_check needs one value per saccade")
    out = [",".join(COLUMNS)]
    for s in range(opc.shape[0]):
        vals = ["%d" % (first + s), "%.6f" % err[s], "" if chk is None else "%.6f" % chk[s]]
        vals += ["%.6f" % opc[s, j] for j in TABLE1_INDEX]
        out.append(",".join(vals))
    return out


def write_csv(path: str, opc, opt_err, cpu_check=None, first: int = 1) -> None:
    with open(path, "w") as f:
        f.write("\n".join(rows(opc, opt_err, cpu_check, first)) + "\n")


def read_csv(path: str):
    """(opc [S][18] in Table 1 order, opt_err [S], cpu_check [S] with NaN where empty)."""
    lines = [l.strip() for l in open(path) if l.strip()]
    if lines[0].split(",") != COLUMNS:
        raise ValueError("not an OPMM result file")
    S = len(lines) - 1
    opc = np.zeros((S, 18))
    err = np.zeros(S)
    chk = np.full(S, np.nan)
    for s, l in enumerate(lines[1:]):
        v = l.split(",")
        err[s] = float(v[1])
        if v[2]:
            chk[s] = float(v[2])
        for c, j in enumerate(TABLE1_INDEX):
            opc[s, j] = float(v[3 + c])
    return opc, err, chk
