"""Pose-difference measures shared by tests and the benchmark (no method arithmetic)."""
import numpy as np


def rot_err_deg(Ta, Tb) -> float:
    """Angle of R_a^T R_b in degrees."""
    dR = np.asarray(Ta)[:3, :3].T @ np.asarray(Tb)[:3, :3]
    c = np.clip((np.trace(dR) - 1.0) / 2.0, -1.0, 1.0)
    # arccos loses precision near 1; use the skew part for small angles.
    s = 0.5 * np.linalg.norm([dR[2, 1] - dR[1, 2], dR[0, 2] - dR[2, 0], dR[1, 0] - dR[0, 1]])
    return float(np.degrees(np.arctan2(s, c)))


def trans_err_m(Ta, Tb) -> float:
    return float(np.linalg.norm(np.asarray(Ta)[:3, 3] - np.asarray(Tb)[:3, 3]))
