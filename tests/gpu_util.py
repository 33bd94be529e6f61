"""Helpers shared by the GPU tests: device copies, the oracle side of a factor, comparisons."""
import numpy as np
import torch

import oracle
from tests.metrics import factor_errors

TOL_FP64_ACC = 1e-5   # FP32 per-point math, FP64 accumulation; FP64 math
TOL_KAHAN = 1e-4      # FP32 per-point math, compensated FP32 accumulation


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def cloud_dev(xyz, cov):
    return dev(np.asarray(xyz, np.float32)), dev(np.asarray(cov, np.float32))


def tol_for(precision):
    import paper_2202_00242_amd.vgicp as V
    return TOL_KAHAN if precision == V.VGICP_ACC_KAHAN_FP32 else TOL_FP64_ACC


def compare_factor(gpu, ref, tol, what=""):
    H = gpu["H"].cpu().numpy()
    b = gpu["b"].cpu().numpy()
    e = float(gpu["err"].cpu().numpy()[0])
    nin = int(gpu["inliers"].cpu().numpy()[0])
    assert nin == ref["inliers"], f"{what}: inliers {nin} vs {ref['inliers']}"
    err = factor_errors(H, b, e, ref["H"], ref["b"], ref["e"])
    assert max(err["H"], err["b"], err["e"]) <= tol, f"{what}: {err}"
    return err


def oracle_factor(txyz, tcov, res, sxyz, scov, Tt, Ts, binary):
    m = oracle.VoxelMap(txyz, tcov, res)
    return m, oracle.linearize(m, sxyz, scov, Tt, Ts, binary)
