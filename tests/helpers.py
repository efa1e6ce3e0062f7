"""Shared helpers of the GPU tests (comparison metrics, tensor transfer)."""
import numpy as np

PARITY_FP64 = 1e-11  # relative, norm-wise and per element against the vector's max


def rel_norm(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m = np.abs(b).max()
    return float(np.abs(a - b).max() / (m if m > 0 else 1.0))


def assert_parity(gpu, ref, tol=PARITY_FP64, what=""):
    rn, rm = rel_norm(gpu, ref), rel_max(gpu, ref)
    print(f"[parity] {what}: rel norm {rn:.2e}, rel max {rm:.2e}", flush=True)
    assert rn <= tol and rm <= tol, f"{what}: rel norm {rn:.3e}, rel max {rm:.3e} > {tol:.1e}"
    return rn, rm
