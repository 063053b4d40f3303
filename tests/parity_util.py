"""Error measures shared by the GPU parity tests (no test functions here).

rel_rms(y) = sqrt(sum_i |y_i - y_ref_i|^2 / sum_i |y_ref_i|^2), vectors and
tensors by their Euclidean/Frobenius norms: the specified bound (1e-5 for
the float32 path).  A relative RMS over millions of particles can hide a
localised defect (ten particles missing one neighbour each move it by
~1e-6), so the tests also bound the worst particle:

    e_i = |y_i - y_ref_i| / (|y_ref_i| + s),   s = RMS_i |y_ref_i|,

max_i e_i <= PER_PARTICLE_FP32 (1e-3; one missing neighbour out of 64
gives ~1.5e-2) or PER_PARTICLE_FP64 (1e-8).  The scale s keeps particles
whose own value nearly cancels (a net force close to zero) from counting
rounding noise of their individual terms as a defect.  Pairs at the gravity
cutoff whose range decision differs between float32 and float64 move a
particle by about 1.5 (eps/r_c)^2 m / r_c^2, below 1e-6 of s here.
"""
import numpy as np

PER_PARTICLE_FP32 = 1e-3
PER_PARTICLE_FP64 = 1e-8


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.sqrt(np.sum(b * b))
    num = np.sqrt(np.sum((a - b) ** 2))
    return num / den if den > 0 else num


def particle_major(key, y):
    """Outputs a_* are stored (3, n); every other output is (n, ...)."""
    y = np.asarray(y, np.float64)
    if key.startswith("a_"):
        y = np.moveaxis(y, -1, 0)
    return y.reshape(y.shape[0], -1) if y.ndim > 1 else y[:, None]


def worst_particle(key, got, ref):
    """(max_i e_i, i) for one output; (0.0, -1) when there are no particles."""
    g, r = particle_major(key, got), particle_major(key, ref)
    if g.shape[0] == 0:
        return 0.0, -1
    d = np.sqrt(np.sum((g - r) ** 2, axis=1))
    rn = np.sqrt(np.sum(r * r, axis=1))
    s = float(np.sqrt(np.mean(rn * rn)))
    e = d / (rn + s) if s > 0 else d
    k = int(np.argmax(e))
    return float(e[k]), k


def degenerate_disagreements(got, ref, sel=None):
    """Particles whose coefficient branch differs between the two sides.
    The GPU returns B = grad B = 0 exactly on the degenerate branch (the
    regular branch gives an exact zero with probability zero); the oracle
    reports its branch per particle."""
    if "degenerate" not in ref or "B" not in got:
        return 0
    B = np.asarray(got["B"])
    if sel is not None:
        B = B[sel]
    gpu_deg = np.all(B.reshape(B.shape[0], -1) == 0.0, axis=1)
    orc_deg = np.asarray(ref["degenerate"]).astype(bool)
    return int(np.sum(gpu_deg != orc_deg))
