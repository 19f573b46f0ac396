"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds random draws only (no discretisation arithmetic): both the
GPU path and the oracle build their right-hand sides from these draws with
their own code.

* ``body_force_modes(r)``: for right-hand side r, 16 separable Fourier modes
  per velocity component, b_c(x) = sum_m a_m prod_d sin(pi k_{m,d} x_d), with
  wavenumbers k_{m,d} uniform in 1..4 and amplitudes a_m = N(0,1) / |k_m|^2,
  followed by a lid speed U ~ U(0.5, 2).
* ``random_vector(n, seed)``: standard-normal FP64 vector.
"""
import numpy as np

SEED_BASE = 231106926


def body_force_modes(r, nmodes=16):
    """(modes, U) for right-hand side r; modes[c] = [(a, (k1, k2, k3)), ...]."""
    rng = np.random.default_rng([SEED_BASE, r])
    modes = []
    for _c in range(3):
        lst = []
        for _m in range(nmodes):
            k = rng.integers(1, 5, size=3)
            a = rng.standard_normal() / float(k @ k)
            lst.append((float(a), tuple(int(v) for v in k)))
        modes.append(lst)
    U = float(rng.uniform(0.5, 2.0))
    return modes, U


def modes_to_arrays(modes):
    """Flatten modes into (amp[3, m], waves[3, m, 3]) arrays."""
    nm = len(modes[0])
    amp = np.zeros((3, nm))
    wav = np.zeros((3, nm, 3), dtype=np.int32)
    for c in range(3):
        for m, (a, k) in enumerate(modes[c]):
            amp[c, m] = a
            wav[c, m] = k
    return amp, wav


def random_vector(n, seed, scale=1.0):
    """Seeded standard-normal FP64 vector of length n."""
    return scale * np.random.default_rng([SEED_BASE, 7, seed]).standard_normal(n)
