"""Closed form of the QPE output state (test infrastructure only).

The QPE circuit of Section IV-A (Eq. 2-3, QPE figure) prepares the counting
register in (1/sqrt N) sum_k e^{2 pi i phi k} |k>, and the inverse QFT maps
|k> to (1/sqrt N) sum_m e^{-2 pi i k m / N} |m>. Hence, with the eigen qubit in
|1>, the amplitude of counting value m is the geometric sum

    alpha_m = (1/N) sum_{k=0}^{N-1} e^{2 pi i k (phi - m/N)}.

Writing N phi = I + f (I integer, 0 <= f < 1) and d = I - m reduced to the
signed range [-N/2, N/2) (the sum only depends on d modulo N),

    alpha_m = sin(pi f) / (N sin(pi (d+f)/N)) * e^{i pi (f - (d+f)/N)},

with alpha_m = 1 when d = f = 0. With the signed d, (d+f)/N is exact and
small near the peak, so sin never loses relative accuracy to cancellation.
The state index of counting value m is m + 2^t (the eigen qubit is bit t);
every other amplitude is 0.
"""
from __future__ import annotations

import math

import numpy as np


def split_phase(t: int, phi: float):
    """(I, f) with 2^t phi = I + f, computed exactly in binary64."""
    x = math.ldexp(phi, t)
    i = math.floor(x)
    return int(i), x - i


def qpe_amplitudes(t: int, phi: float, m) -> np.ndarray:
    """alpha_m for the counting values m (int array); complex128."""
    N = 1 << t
    I, f = split_phase(t, phi)
    m = np.asarray(m, dtype=np.int64)
    d = np.mod(I - m + N // 2, N) - N // 2
    d = d.astype(np.float64)
    u = (d + f) / N
    num = math.sin(math.pi * f)
    with np.errstate(divide="ignore", invalid="ignore"):
        mag = num / (N * np.sin(np.pi * u))
    ang = np.pi * (f - u)
    out = mag * np.exp(1j * ang)
    exact = (d == 0) & (f == 0.0)
    out[exact] = 1.0
    if f == 0.0:
        out[~exact] = 0.0
    return out


def qpe_state(n: int, phi: float) -> np.ndarray:
    """The full final state (2^n complex128) of the n-qubit QPE circuit."""
    t = n - 1
    s = np.zeros(1 << n, dtype=np.complex128)
    s[(1 << t):] = qpe_amplitudes(t, phi, np.arange(1 << t))
    return s


def qpe_probabilities(t: int, phi: float, m) -> np.ndarray:
    return np.abs(qpe_amplitudes(t, phi, m)) ** 2


def qpe_argmax(t: int, phi: float) -> int:
    """round(N phi) mod N, the most likely counting value (f = 1/2 is a tie)."""
    I, f = split_phase(t, phi)
    return int((I + (1 if f > 0.5 else 0)) % (1 << t))
