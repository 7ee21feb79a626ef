"""Rounding of oracle inputs to the library's storage formats.

Reduced-precision parity compares the GPU with the oracle evaluated on the
same quantised inputs: links keep their first two rows in the storage type
and rebuild the third as conj(row0 x row1); the clover blocks keep the real
diagonal and the upper triangle of each 6x6 chirality block (the lower
triangle is its conjugate); spinors are rounded to complex64.  These helpers
only round numbers; they hold none of the solver's arithmetic.
"""

import numpy as np
import torch


def round_real(x: np.ndarray, kind: str) -> np.ndarray:
    """Round float64 values to 'f64', 'f32', 'f16' or 'bf16' (via float32, RNE)."""
    x = np.asarray(x, dtype=np.float64)
    if kind == "f64":
        return x.copy()
    f = x.astype(np.float32)
    if kind == "f32":
        return f.astype(np.float64)
    t = torch.from_numpy(f)
    if kind == "f16":
        return t.to(torch.float16).to(torch.float64).numpy()
    if kind == "bf16":
        return t.to(torch.bfloat16).to(torch.float64).numpy()
    raise ValueError(kind)


def round_complex(z: np.ndarray, kind: str) -> np.ndarray:
    return round_real(z.real, kind) + 1j * round_real(z.imag, kind)


def quantise_links(U: np.ndarray, kind: str) -> np.ndarray:
    if kind == "f64":
        return U.copy()
    r0 = round_complex(U[..., 0, :], kind)
    r1 = round_complex(U[..., 1, :], kind)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def quantise_clover(Am: np.ndarray, kind: str) -> np.ndarray:
    """Round per-site 12x12 clover matrices the way the packed storage does."""
    if kind == "f64":
        return Am.copy()
    out = np.zeros_like(Am)
    iu = np.triu_indices(6, 1)
    for h in range(2):
        blk = Am[:, 6 * h:6 * h + 6, 6 * h:6 * h + 6]
        q = np.zeros_like(blk)
        d = round_real(np.real(np.diagonal(blk, axis1=1, axis2=2)), kind)
        q[:, np.arange(6), np.arange(6)] = d
        up = 0.5 * (blk[:, iu[0], iu[1]] + np.conj(blk[:, iu[1], iu[0]]))
        up = round_complex(up, kind)
        q[:, iu[0], iu[1]] = up
        q[:, iu[1], iu[0]] = np.conj(up)
        out[:, 6 * h:6 * h + 6, 6 * h:6 * h + 6] = q
    return out


def quantise_spinor_f16(x: np.ndarray) -> np.ndarray:
    """FP16 spinor storage with a per-site power-of-two scale: per site the
    largest |re| or |im| m (taken in FP32) = f 2^e with f in [0.5, 1); the
    site is divided by 2^(e - 15), rounded to FP16 (round to nearest even)
    and multiplied back.  Sites with m < 2^-112 are stored as zero.  Input
    [..., V, 4, 3] complex; the scaling is exact, so this reproduces the
    stored values bit for bit."""
    z = np.asarray(x).astype(np.complex64)
    shp = z.shape
    re = z.real.reshape(shp[:-2] + (12,))
    im = z.imag.reshape(shp[:-2] + (12,))
    m = np.maximum(np.abs(re).max(axis=-1), np.abs(im).max(axis=-1)).astype(np.float32)
    _, e = np.frexp(m)
    nz = m >= np.float32(2.0 ** -112)
    sc = np.where(nz, np.ldexp(np.float32(1.0), (e - 15)).astype(np.float32), np.float32(0.0))
    inv = np.where(nz, np.ldexp(np.float32(1.0), (15 - e)).astype(np.float32), np.float32(0.0))
    qr = (re * inv[..., None]).astype(np.float16).astype(np.float32) * sc[..., None]
    qi = (im * inv[..., None]).astype(np.float16).astype(np.float32) * sc[..., None]
    return (qr.astype(np.float64) + 1j * qi.astype(np.float64)).reshape(shp)


STORAGE_KIND = {0: "f64", 1: "f32", 2: "f16", 3: "bf16"}
CLOVER_KIND = {0: "f64", 1: "f32", 2: "f16", 3: "f16"}
