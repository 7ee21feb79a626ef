"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generation only: random numbers, SU(3) link
matrices drawn from a Gaussian Lie-algebra element, complex-Gaussian spinor
fields, point/Z2 sources and lattice bookkeeping.  It contains none of the
solver's arithmetic (no Dirac operator, no clover term, no Krylov step).

Conventions (the paper, section 2.2, names the operator but fixes none of
these; they are the readings listed in the design notes):

* lattice extents ``dims = (T, X, Y, Z)``; direction mu = 0 is time;
* lexicographic site index ``i = z + Z*(y + Y*(x + X*t))``;
* gauge links ``U[i, mu, a, b]`` complex128, ``U_mu(x)`` connects x to x+mu;
* spinors ``psi[rhs, i, spin, colour]`` complex128;
* spin-colour index ``sc = 3*spin + colour``.

Random numbers come from a counter-based generator: the n-th output of
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) for a 64-bit key, so any entry can be produced
independently of the others.  ``sm64(key, n)`` is that output;
``stream_key(seed, stream)`` derives the key of a named stream as
``sm64(seed, stream)``.  Uniforms are ``(x >> 11) * 2**-53`` and Gaussians
use Box-Muller on consecutive pairs.  The HIP library implements the same
published generator on the device for the random fields it draws itself.
"""

from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Named random streams (the stream index feeds stream_key).
STREAM_GAUGE = 1
STREAM_SPINOR = 2
STREAM_GAUGE_TRANSFORM = 3
STREAM_SITE = 4
STREAM_DFL = 5   # deflation-field seeds drawn by the method itself
STREAM_Z2 = 6    # Z2-noise sources drawn by the method itself


def _parallel_chunks(fn, starts):
    """Run fn over chunk offsets on a thread pool (numpy releases the GIL)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    starts = list(starts)
    nw = max(1, min(len(starts), os.cpu_count() or 1, 16))
    if nw == 1:
        for s in starts:
            fn(s)
        return
    with ThreadPoolExecutor(nw) as ex:
        list(ex.map(fn, starts))


def _u64(x):
    return np.asarray(x, dtype=np.uint64)


def sm64(key, n):
    """n-th SplitMix64 output (n = 0, 1, ...) for state ``key``; vectorised."""
    with np.errstate(over="ignore"):
        z = _u64(key) + (_u64(n) + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def stream_key(seed: int, stream: int) -> np.uint64:
    return np.uint64(sm64(np.uint64(seed), np.uint64(stream)))


def uniform(key, n):
    """Uniform in [0, 1) from 53 high bits."""
    return (sm64(key, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian(key, j):
    """Standard normal number j of the stream: Box-Muller on outputs 2k, 2k+1.

    Even j takes the cosine branch, odd j the sine branch of pair k = j // 2.
    """
    j = _u64(j)
    k = j >> np.uint64(1)
    u1 = 1.0 - uniform(key, np.uint64(2) * k)          # (0, 1]
    u2 = uniform(key, np.uint64(2) * k + np.uint64(1))
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return np.where((j & np.uint64(1)) == 0, r * np.cos(ang), r * np.sin(ang))


# --------------------------------------------------------------------------
# Lattice bookkeeping
# --------------------------------------------------------------------------

def volume(dims) -> int:
    T, X, Y, Z = dims
    return int(T) * int(X) * int(Y) * int(Z)


def lex(dims, t, x, y, z):
    T, X, Y, Z = dims
    return z + Z * (y + Y * (x + X * t))


def coords(dims, i):
    """Inverse of ``lex``: returns (t, x, y, z)."""
    T, X, Y, Z = dims
    i = np.asarray(i)
    z = i % Z
    y = (i // Z) % Y
    x = (i // (Z * Y)) % X
    t = i // (Z * Y * X)
    return t, x, y, z


def seeded_site(dims, seed: int):
    """A site drawn uniformly from the lattice (used for point sources)."""
    key = stream_key(seed, STREAM_SITE)
    V = volume(dims)
    return int(min(int(uniform(key, 0) * V), V - 1))


# --------------------------------------------------------------------------
# SU(3) links from a Gaussian Lie-algebra element
# --------------------------------------------------------------------------

def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_a, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1] = -1j
    l[1, 1, 0] = 1j
    l[2, 0, 0] = 1
    l[2, 1, 1] = -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2] = -1j
    l[4, 2, 0] = 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2] = -1j
    l[6, 2, 1] = 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def reunitarise(U: np.ndarray) -> np.ndarray:
    """Gram-Schmidt the first two rows, third row = conj(row0 x row1).

    The result is in SU(3) to rounding, and its third row is exactly the one
    a reconstruct-12 storage scheme rebuilds from the first two.
    """
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def expi_traceless_hermitian(Q: np.ndarray) -> np.ndarray:
    """exp(i Q) for traceless Hermitian 3x3 matrices Q[..., 3, 3].

    Cayley-Hamilton form exp(iQ) = f0 + f1 Q + f2 Q^2 with the coefficients
    of Morningstar and Peardon (Phys. Rev. D 69 (2004) 054501, eqs. 29-36):
    c0 = det Q, c1 = tr(Q^2)/2, theta = arccos(c0 / c0max),
    u = sqrt(c1/3) cos(theta/3), w = sqrt(c1) sin(theta/3), and for c0 < 0
    the coefficients of -Q with f_j(-c0) = (-1)^j conj(f_j(c0)).  Elementwise
    array operations only (no per-matrix library loop).
    """
    Q2 = Q @ Q
    c1 = 0.5 * np.real(np.trace(Q2, axis1=-2, axis2=-1))
    c0 = np.real(np.trace(Q2 @ Q, axis1=-2, axis2=-1)) / 3.0
    neg = c0 < 0
    c0a = np.abs(c0)
    c0max = 2.0 * (c1 / 3.0) ** 1.5
    ratio = np.where(c0max > 0, c0a / np.where(c0max > 0, c0max, 1.0), 0.0)
    theta = np.arccos(np.clip(ratio, -1.0, 1.0))
    u = np.sqrt(c1 / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(c1) * np.sin(theta / 3.0)
    w2 = w * w
    small = np.abs(w) < 0.05
    xi0 = np.where(small, 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)),
                   np.sin(w) / np.where(small, 1.0, w))
    e2iu = np.exp(2j * u)
    emiu = np.exp(-1j * u)
    cw = np.cos(w)
    u2 = u * u
    h0 = (u2 - w2) * e2iu + emiu * (8.0 * u2 * cw + 2j * u * (3.0 * u2 + w2) * xi0)
    h1 = 2.0 * u * e2iu - emiu * (2.0 * u * cw - 1j * (3.0 * u2 - w2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9.0 * u2 - w2
    tiny = den < 1e-300
    den = np.where(tiny, 1.0, den)
    f0 = np.where(tiny, 1.0, h0 / den)
    f1 = np.where(tiny, 1j, h1 / den)
    f2 = np.where(tiny, -0.5, h2 / den)
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    eye = np.eye(3, dtype=np.complex128)
    return f0[..., None, None] * eye + f1[..., None, None] * Q + f2[..., None, None] * Q2


def su3_from_gaussian(omega: np.ndarray, eps: float) -> np.ndarray:
    """U = exp(i eps H), H = sum_a omega_a lambda_a / 2, for omega[..., 8]."""
    lam = gell_mann()
    sh = omega.shape[:-1]
    H = (omega.reshape(-1, 8).astype(np.complex128) @ lam.reshape(8, 9)).reshape(sh + (3, 3)) * 0.5
    H = 0.5 * (H + np.conj(np.swapaxes(H, -1, -2)))
    return reunitarise(expi_traceless_hermitian(eps * H))


def gauge_field(dims, eps: float, seed: int = 1, progress=None) -> np.ndarray:
    """Synthetic gauge field U[V, 4, 3, 3] with U = exp(i eps H) per link.

    Draw order of the 8 Gaussians: site (lexicographic), then mu, then a.
    Links are periodic in every direction; the fermion boundary phase is
    not part of the field.  progress(fraction) is called now and then.
    """
    import threading
    V = volume(dims)
    key = stream_key(seed, STREAM_GAUGE)
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    chunk = 1 << 16
    nchunks = (V + chunk - 1) // chunk
    done = [0]
    lock = threading.Lock()

    def work(s0):
        s1 = min(V, s0 + chunk)
        j = np.arange(s0 * 32, s1 * 32, dtype=np.uint64)
        om = gaussian(key, j).reshape(s1 - s0, 4, 8)
        out[s0:s1] = su3_from_gaussian(om, eps)
        if progress is not None:
            with lock:
                done[0] += 1
                if done[0] % 16 == 0:
                    progress(done[0] / nchunks)

    _parallel_chunks(work, range(0, V, chunk))
    return out


def random_su3_field(V: int, seed: int, eps: float = 2.0) -> np.ndarray:
    """Per-site random SU(3) matrices Omega[V, 3, 3] (for gauge transforms)."""
    key = stream_key(seed, STREAM_GAUGE_TRANSFORM)
    om = gaussian(key, np.arange(V * 8, dtype=np.uint64)).reshape(V, 8)
    return su3_from_gaussian(om, eps)


def plaquette(dims, U: np.ndarray) -> float:
    """Average of Re tr U_p / 3 over all plaquettes (a field fingerprint)."""
    T, X, Y, Z = dims
    Ul = U.reshape(T, X, Y, Z, 4, 3, 3)
    tot = 0.0
    n = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = Ul[..., mu, :, :]
            b = np.roll(Ul[..., nu, :, :], -1, axis=mu)
            c = np.roll(Ul[..., mu, :, :], -1, axis=nu)
            d = Ul[..., nu, :, :]
            p = a @ b @ np.conj(np.swapaxes(c, -1, -2)) @ np.conj(np.swapaxes(d, -1, -2))
            tot += np.real(np.trace(p, axis1=-2, axis2=-1)).sum() / 3.0
            n += p.shape[0] * p.shape[1] * p.shape[2] * p.shape[3]
    return tot / n


# --------------------------------------------------------------------------
# Spinor fields and sources
# --------------------------------------------------------------------------

def gaussian_spinor(dims, nrhs: int = 1, seed: int = 1001) -> np.ndarray:
    """Complex-Gaussian spinors psi[nrhs, V, 4, 3], unit variance per real part."""
    V = volume(dims)
    key = stream_key(seed, STREAM_SPINOR)
    n = nrhs * V * 12
    out = np.empty(n, dtype=np.complex128)
    chunk = 1 << 22
    for s0 in range(0, n, chunk):
        s1 = min(n, s0 + chunk)
        j = np.arange(2 * s0, 2 * s1, dtype=np.uint64)
        g = gaussian(key, j)
        out[s0:s1] = g[0::2] + 1j * g[1::2]
    return out.reshape(nrhs, V, 4, 3)


def point_source(dims, site: int, sc: int) -> np.ndarray:
    """eta(x) = delta_{x, site} delta_{spin-colour, sc}, shape [V, 4, 3]."""
    V = volume(dims)
    eta = np.zeros((V, 4, 3), dtype=np.complex128)
    eta[site, sc // 3, sc % 3] = 1.0
    return eta


def z2_source(dims, seed: int, index: int = 0) -> np.ndarray:
    """Real +-1 noise on every component of every site, shape [V, 4, 3].

    Component j = 12*site + sc of noise vector ``index`` takes the sign of
    the top bit of sm64(stream_key(seed, Z2), index*12*V + j).
    """
    V = volume(dims)
    key = stream_key(seed, STREAM_Z2)
    j = np.arange(V * 12, dtype=np.uint64) + np.uint64(index * 12 * V)
    bits = sm64(key, j) >> np.uint64(63)
    return (1.0 - 2.0 * bits.astype(np.float64)).astype(np.complex128).reshape(V, 4, 3)


def shift_field(dims, f: np.ndarray, g) -> np.ndarray:
    """Translate a site field: out(x + g) = f(x), for f[V, ...]."""
    T, X, Y, Z = dims
    sh = f.reshape((T, X, Y, Z) + f.shape[1:])
    sh = np.roll(sh, shift=tuple(int(v) for v in g), axis=(0, 1, 2, 3))
    return sh.reshape(f.shape)
