"""FP64 CPU oracle for the display-side steps after the hologram: double-phase amplitude
coding (DPAC) of the complex SLM field and angular-spectrum focal stacks.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/`` and never by
the product library, with which it shares no code.

* DPAC (Sec. 5, phase-only encoding, and the supplement's display section).  The printed
  pair of phases is garbled; the reading taken is the standard double-phase form of the
  works the paper cites (Hsueh and Sawchuk 1978; Maimone et al. 2017): a field value
  a e^{j phi} with a <= a_max is the mean of two unit phasors,
      a e^{j phi} = a_max (e^{j P-} + e^{j P+}) / 2,   P-/+ = phi -/+ arccos(a / a_max),
  and the two phases are interlaced like a checkerboard: P- where n_x + n_y is even, P+
  where it is odd.  a_max defaults to the largest |u| of each wavelength channel; a ratio
  a / a_max above 1 (a caller-chosen a_max that is too small) is clipped to 1.  An all-zero
  channel has a_max = 0 and is encoded with ratio 0.  Phases are not wrapped: P lies in
  (-2 pi, 2 pi].
* Half-band Fourier filter.  The checkerboard moves the unwanted half of the encoding to the
  Nyquist corner of the spectrum; the filter keeps the frequencies with |m'_x| < N_x / 4 and
  |m'_y| < N_y / 4 (signed FFT indices), half of the band along each axis.
* Focal stack.  The angular-spectrum method of Eq. 3-4 on the periodic grid of the hologram:
      P(u; d) = IDFT( DFT(u) H(nu, d) ),   H(nu, d) = exp(j 2 pi d sqrt(1/lambda^2 - |nu|^2))
  inside the propagating band and 0 outside.  A Gaussian whose hologram term carries
  H(nu, -z) (Eq. 5, 12) is in focus in the plane d = z.  The stack is |P(u; d_k)|^2 per
  plane and wavelength, or the complex fields themselves.
"""
from __future__ import annotations

import math

import numpy as np

from . import signed_freq_index
from .exact import transfer


def channel_amax(u: np.ndarray) -> np.ndarray:
    """Largest |u| of each wavelength channel of a (C, ny, nx) field."""
    return np.abs(u).reshape(u.shape[0], -1).max(axis=1)


def dpac_phases(u: np.ndarray, a_max=None):
    """The two double-phase phases (P-, P+) of every pixel of a (C, ny, nx) field."""
    u = np.asarray(u, dtype=np.complex128)
    C = u.shape[0]
    am = channel_amax(u) if a_max is None else np.broadcast_to(np.asarray(a_max, dtype=np.float64), (C,))
    a = np.abs(u)
    r = np.zeros_like(a)
    for c in range(C):
        if am[c] > 0.0:
            r[c] = np.clip(a[c] / am[c], 0.0, 1.0)
    theta = np.arccos(r)
    phi = np.angle(u)
    return phi - theta, phi + theta


def checkerboard(ny: int, nx: int) -> np.ndarray:
    """True where n_x + n_y is even."""
    return (np.add.outer(np.arange(ny), np.arange(nx)) % 2) == 0


def dpac_encode(u: np.ndarray, a_max=None) -> np.ndarray:
    """The interlaced phase-only pattern: P- on even pixels (n_x + n_y even), P+ on odd."""
    pm, pp = dpac_phases(u, a_max)
    even = checkerboard(u.shape[-2], u.shape[-1])
    return np.where(even[None], pm, pp)


def half_band_mask(grid) -> np.ndarray:
    """1 where |m'_x| < N_x / 4 and |m'_y| < N_y / 4, in FFT order."""
    mx = np.abs(signed_freq_index(grid.nx)) * 4 < grid.nx
    my = np.abs(signed_freq_index(grid.ny)) * 4 < grid.ny
    return (my[:, None] & mx[None, :]).astype(np.float64)


def propagate(u: np.ndarray, grid, d: float, half_band: bool = False) -> np.ndarray:
    """P(u; d) for every wavelength channel of a (C, ny, nx) field, optionally through the
    half-band filter."""
    u = np.asarray(u, dtype=np.complex128)
    out = np.empty_like(u)
    mask = half_band_mask(grid) if half_band else 1.0
    for c, lam in enumerate(grid.lambdas):
        out[c] = np.fft.ifft2(np.fft.fft2(u[c]) * transfer(grid, lam, d) * mask)
    return out


def focal_stack(inp: np.ndarray, grid, depths, phase_input: bool = False, half_band: bool = False,
                complex_output: bool = False) -> np.ndarray:
    """(K, C, ny, nx): |P(u; d_k)|^2 for each depth d_k (or the fields with complex_output).
    With phase_input the input is a phase-only pattern P and u = e^{j P}."""
    u = np.exp(1j * np.asarray(inp, dtype=np.float64)) if phase_input else np.asarray(inp, dtype=np.complex128)
    planes = [propagate(u, grid, float(d), half_band) for d in depths]
    st = np.stack(planes) if planes else np.zeros((0,) + u.shape, dtype=np.complex128)
    return st if complex_output else np.abs(st) ** 2


def phase_distance(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """|p - q| reduced modulo 2 pi to [0, pi]."""
    d = np.mod(np.asarray(p, dtype=np.float64) - np.asarray(q, dtype=np.float64), 2.0 * math.pi)
    return np.minimum(d, 2.0 * math.pi - d)
