"""Independent closed forms that pin the oracle (and, through it, the GPU path).

None of these calls the oracle or the HIP library.  Each reaches the result of
the stencil definition (Section 1: a point at step t+1 is a weighted sum of the
(2r+1)-per-direction neighbourhood at step t; Section 3.3: Jacobi update) by a
different mathematical route:

* ``ndimage_sweep``  -- scipy's N-d correlation filter applied T times
  (zero halo = constant mode with 0, periodic = grid-wrap mode);
* ``fft_sweep``      -- periodic grids are diagonalised by the DFT; the shift
  u[x+o] has symbol exp(+2*pi*i*k.o/N), so u_T = IFFT(sigma^T FFT(u_0));
* ``dst_sweep``      -- zero-halo grids with r = 1 and weights symmetric under
  every axis reflection are diagonalised by DST-I with eigenvalue
  sum_j c_j prod_i cos(pi*k_i*o_ji/(N_i+1));
* ``fft_adjoint``    -- the periodic adjoint in Fourier space:
  dL/du0 = IFFT(conj(sigma)^T FFT(g)), and
  dL/dc_j = sum_t <lambda_{t+1}, S_j u_t>
          = (1/n) Re sum_k conj(Lhat_k) * e_j(k) * sigma(k)^{T-1} * T * uhat_k
  (all lambda_{t+1}, u_t share the Fourier basis, so each of the T terms
  equals the same expression).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.fft
import scipy.ndimage


def canonical_offsets(dim: int, r: int, kind: int) -> np.ndarray:
    """Offsets in lexicographic order of the tuple (axis 0 most significant),
    filtered to the star (at most one non-zero component) or the box."""
    out = []
    for o in itertools.product(range(-r, r + 1), repeat=dim):
        if kind == 0 and sum(1 for v in o if v != 0) > 1:
            continue
        out.append(o)
    return np.array(out, dtype=np.int64).reshape(-1, dim)


def weight_array(offs: np.ndarray, coeffs, r: int) -> np.ndarray:
    dim = offs.shape[1]
    w = np.zeros((2 * r + 1,) * dim)
    for o, c in zip(offs, coeffs):
        w[tuple(int(v) + r for v in o)] += c
    return w


def ndimage_sweep(u0, offs, coeffs, r, bc, T):
    w = weight_array(np.asarray(offs), coeffs, r)
    u = np.array(u0, dtype=np.float64)
    mode = "grid-wrap" if bc == 1 else "constant"
    for _ in range(T):
        u = scipy.ndimage.correlate(u, w, mode=mode, cval=0.0)
    return u


def symbol(shape, offs, coeffs) -> np.ndarray:
    """sigma(k) = sum_j c_j exp(+2 pi i sum_i k_i o_ji / N_i) on the full DFT grid."""
    grids = np.meshgrid(*[np.fft.fftfreq(n) * n for n in shape], indexing="ij")
    s = np.zeros(tuple(shape), dtype=np.complex128)
    for o, c in zip(offs, coeffs):
        phase = sum(2j * np.pi * k * int(oi) / n for k, oi, n in zip(grids, o, shape))
        s += c * np.exp(phase)
    return s


def fft_sweep(u0, offs, coeffs, T):
    u0 = np.asarray(u0, dtype=np.float64)
    s = symbol(u0.shape, offs, coeffs)
    return np.real(np.fft.ifftn(s ** T * np.fft.fftn(u0)))


def dst_sweep(u0, offs, coeffs, T):
    u0 = np.asarray(u0, dtype=np.float64)
    shape = u0.shape
    grids = np.meshgrid(*[np.arange(1, n + 1) for n in shape], indexing="ij")
    lam = np.zeros(shape)
    for o, c in zip(offs, coeffs):
        term = np.full(shape, c)
        for k, oi, n in zip(grids, o, shape):
            term = term * np.cos(np.pi * k * int(oi) / (n + 1))
        lam += term
    return scipy.fft.idstn(lam ** T * scipy.fft.dstn(u0, type=1), type=1)


def fft_adjoint(u0, g, offs, coeffs, T):
    """(dL/du0, dL/dc) of L with dL/du_T = g, for a periodic grid."""
    u0 = np.asarray(u0, dtype=np.float64)
    n = u0.size
    s = symbol(u0.shape, offs, coeffs)
    uh = np.fft.fftn(u0)
    gh = np.fft.fftn(np.asarray(g, dtype=np.float64))
    grad_u0 = np.real(np.fft.ifftn(np.conj(s) ** T * gh))
    grids = np.meshgrid(*[np.fft.fftfreq(m) * m for m in u0.shape], indexing="ij")
    grad_c = np.zeros(len(coeffs))
    if T > 0:
        # lambda_{t+1} has Fourier coefficients conj(s)^{T-1-t} gh and u_t has
        # s^t uh; by Parseval <lambda, S_j u> = (1/n) sum_k conj(lam_k) e_j(k) u_k,
        # and conj(conj(s)^{T-1-t}) s^t = s^{T-1}: every step contributes the same.
        base = np.conj(gh) * s ** (T - 1) * uh
        for j, o in enumerate(offs):
            e = np.exp(sum(2j * np.pi * k * int(oi) / m for k, oi, m in zip(grids, o, u0.shape)))
            grad_c[j] = T * np.real(np.sum(base * e)) / n
    return grad_u0, grad_c


def loss_grad(u_T, y):
    return np.asarray(u_T) - np.asarray(y)
