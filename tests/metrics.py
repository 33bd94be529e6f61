"""Scale-free error metric for a Gauss-Newton factor (H, b, e) against a reference.

  eps_H = max_ij |dH_ij| / sqrt(H_ii H_jj)
  eps_b = max_i  |db_i|  / sqrt(H_ii e)        (|b_i| <= sqrt(H_ii e) by Cauchy-Schwarz)
  eps_e = |de| / e

H_ii, H_jj and e are the reference's. Zero denominators (zero inliers) compare absolutely.
"""
import numpy as np


def factor_errors(H, b, e, H_ref, b_ref, e_ref):
    H = np.asarray(H, dtype=np.float64)
    H_ref = np.asarray(H_ref, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    b_ref = np.asarray(b_ref, dtype=np.float64)
    dim = H_ref.shape[-1]
    H = H.reshape(dim, dim)
    H_ref = H_ref.reshape(dim, dim)
    diag = np.clip(np.diag(H_ref), 0.0, None)
    den_H = np.sqrt(np.outer(diag, diag))
    dH = np.abs(H - H_ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        eH = np.where(den_H > 0, dH / den_H, dH)
        den_b = np.sqrt(diag * max(float(e_ref), 0.0))
        eb = np.where(den_b > 0, np.abs(b - b_ref) / den_b, np.abs(b - b_ref))
    ee = abs(float(e) - float(e_ref)) / e_ref if e_ref > 0 else abs(float(e) - float(e_ref))
    fro = np.linalg.norm(H - H_ref) / max(np.linalg.norm(H_ref), 1e-300)
    return {"H": float(eH.max()), "b": float(eb.max()), "e": float(ee), "H_fro": float(fro)}


def max_factor_error(errs):
    return max(errs["H"], errs["b"], errs["e"])
