"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle)."""
import numpy as np

import oracle

# Tolerance (spec: 1e-4 relative per pixel and per gradient entry, FP32
# GPU vs FP64 oracle). Absolute floors derived from the arithmetic:
#  - IMG_FLOOR: one FP32 ulp of the largest pixel (values are means of
#    non-negative radiances, no cancellation);
#  - GRAD_MASS: a gradient entry is a sum of many signed contributions (FP32
#    atomics in any order), so its rounding error is bounded by the
#    per-contribution relative error times the sum of their magnitudes
#    ("mass", computed by the oracle in FP64; a boundary sample's weight is a
#    difference f+ - f-, whose error scales with |f+| + |f-|). The longest
#    FP32 chain in a contribution is the edge-tree pdf: a product of up to ~27
#    level probabilities, each from ~25 FP32 operations, i.e. ~650 u32
#    (u32 = 6e-8) -> 4e-5.
REL = 1e-4
IMG_FLOOR = 1.2e-7
GRAD_MASS = 4e-5
# the plain reading of "1e-4 relative": 1e-4 |orc| + 1e-7 max |orc| (one FP32
# ulp of the largest entry); every comparison reports how many entries pass
# under it alone and how many need the rounding-scale term above
RULE_T_FLOOR = 1e-7

# one line per comparison, printed at the end of the session (conftest)
SUMMARY = []


def oracle_reference(scene, cam, spp, depth, seed, dimg, threads=8, **kw):
    r = oracle.render(scene, cam, spp, depth, seed, d_image=dimg, want_flags=True, exclude_flagged=True,
                      threads=threads, **kw)
    r["mask"] = (1 - r["unit_flags"]).astype(np.uint8)
    return r


def compare(name, gpu, orc, mass=None, floor_rel=IMG_FLOOR, case=""):
    gpu = np.asarray(gpu, np.float64).ravel()
    orc = np.asarray(orc, np.float64).ravel()
    amax = np.abs(orc).max() if orc.size else 0.0
    tol = REL * np.abs(orc) + floor_rel * amax
    tol_t = REL * np.abs(orc) + RULE_T_FLOOR * amax
    if mass is not None:
        tol = tol + GRAD_MASS * np.asarray(mass, np.float64).ravel()
    err = np.abs(gpu - orc)
    in_t = err <= tol_t
    extra = ~in_t & (err <= tol)
    line = f"{case} {name}: {int(in_t.sum())}/{gpu.size} within rule T"
    if extra.any():
        # share of the allowance beyond rule T (the rounding-scale term, and the
        # floor's excess over one FP32 ulp of the largest entry) that they use
        used = float(((err - tol_t)[extra] / np.maximum((tol - tol_t)[extra], 1e-300)).max())
        line += f", {int(extra.sum())} need the rounding-scale term (using at most {used:.2f} of it)"
    SUMMARY.append(line)
    bad = np.nonzero(err > tol)[0]
    if bad.size:
        worst = bad[np.argsort(-(err[bad] / np.maximum(tol[bad], 1e-300)))[:8]]
        lines = [f"{name}: {bad.size}/{gpu.size} entries outside tolerance"]
        for i in worst:
            extra = f" mass={mass.ravel()[i]:.3e}" if mass is not None else ""
            lines.append(f"  [{i}] gpu={gpu[i]:.9e} orc={orc[i]:.9e} err={err[i]:.3e} tol={tol[i]:.3e}{extra}")
        raise AssertionError("\n".join(lines))
    return float((err / np.maximum(np.abs(orc), 1e-30)).max()) if orc.size else 0.0
