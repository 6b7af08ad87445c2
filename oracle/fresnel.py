"""Point-source object wave, Fresnel form, as a direct 2D sum (oracle).

Paper, Sec. 2, Eq. 1: the hologram is the superposition over object points i of
A_i / r_i * exp(j k r_i).  The hot path uses the paraxial (Fresnel) form of that
sum, whose kernel depends only on the lateral offset:

    O(x, y) = sum_i A_i * exp( i*pi * pitch^2 * ((x - x_i)^2 + (y - y_i)^2) / (lambda * z) )

Readings (the specification table of the paper is missing): object and hologram
share one grid of pixel pitch ``pitch``, aligned index to index, so every offset
is an integer number of pixels; the fringe covers the whole hologram plane (no
truncation, no band limit, no wrap-around).  Optionally each layer carries the
constant paraxial prefactor exp(i k z) / z of Eq. 1 (k = 2 pi / lambda).

This module does NOT use separability: every (point, pixel) term evaluates the
2D exponent itself.  Work is split over pixel chunks only.
"""

import os
from multiprocessing import get_context

import numpy as np


def phase_2d(dy, dx, lam, pitch, z):
    """pi pitch^2 (dx^2 + dy^2) / (lambda z) for integer pixel offsets (radians)."""
    dy = np.asarray(dy, dtype=np.float64)
    dx = np.asarray(dx, dtype=np.float64)
    return np.pi * pitch * pitch * (dx * dx + dy * dy) / (lam * z)


def kernel_2d(dy, dx, lam, pitch, z):
    """exp(i pi pitch^2 (dx^2 + dy^2) / (lambda z)) for integer pixel offsets."""
    th = phase_2d(dy, dx, lam, pitch, z)
    return np.cos(th) + 1j * np.sin(th)


def prefactor(lam, z):
    """Constant of Eq. 1's paraxial expansion for a layer at distance z."""
    return np.exp(1j * 2.0 * np.pi * z / lam) / z


def _chunk_sum(args):
    ys, xs, qs, ps, amps, lam, pitch, z = args
    out = np.zeros(ys.shape[0], dtype=np.complex128)
    # work in blocks of ~256k terms (pixels x points) to stay cache- and allocator-friendly
    pstep = min(qs.shape[0], 131072)
    step = max(1, 131072 // pstep)
    a_re = np.ascontiguousarray(np.real(amps))
    a_im = np.ascontiguousarray(np.imag(amps)) if np.iscomplexobj(amps) else None
    for s in range(0, ys.shape[0], step):
        for t in range(0, qs.shape[0], pstep):
            th = phase_2d(ys[s:s + step, None] - qs[None, t:t + pstep],
                          xs[s:s + step, None] - ps[None, t:t + pstep], lam, pitch, z)
            # sum_i a_i exp(i th_i) with exp(i th) = cos th + i sin th
            c, sn = np.cos(th), np.sin(th)
            ar = a_re[t:t + pstep]
            if a_im is None:
                out[s:s + step] += c @ ar + 1j * (sn @ ar)
            else:
                ai = a_im[t:t + pstep]
                out[s:s + step] += (c @ ar - sn @ ai) + 1j * (c @ ai + sn @ ar)
    return out


def worker_count():
    """Processes for the direct sum: the host's CPU share, at most 16.

    ``ORACLE_WORKERS`` overrides it (GPU test runs keep the pool small).
    """
    env = os.environ.get("ORACLE_WORKERS")
    if env:
        return max(1, int(env))
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


_SHARED = None  # (ys, xs, qs, ps, amps, lam, pitch, z) inherited by forked workers


def _shared_chunk(bounds):
    a, b = bounds
    ys, xs, qs, ps, amps, lam, pitch, z = _SHARED
    try:  # one BLAS thread per worker process: the pool already fills the cores
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        return _chunk_sum((ys[a:b], xs[a:b], qs, ps, amps, lam, pitch, z))
    with threadpool_limits(limits=1):
        return _chunk_sum((ys[a:b], xs[a:b], qs, ps, amps, lam, pitch, z))


def direct_sum(amp, lam, pitch, z, ys, xs, workers=None):
    """Hologram values at pixels (ys[k], xs[k]) of the object field ``amp``.

    ``amp`` is a real or complex (ny, nx) array of point amplitudes on the
    pixel grid; returns complex128 of len(ys).  Points with zero amplitude
    contribute nothing and are skipped.
    """
    global _SHARED
    amp = np.asarray(amp)
    amp = amp.astype(np.complex128 if np.iscomplexobj(amp) else np.float64)
    qs, ps = np.nonzero(amp)
    amps = amp[qs, ps]
    qs = qs.astype(np.float64)
    ps = ps.astype(np.float64)
    ys = np.asarray(ys, dtype=np.float64).ravel()
    xs = np.asarray(xs, dtype=np.float64).ravel()
    if ys.shape[0] == 0 or qs.shape[0] == 0:
        return np.zeros(ys.shape[0], dtype=np.complex128)
    workers = worker_count() if workers is None else workers
    terms = ys.shape[0] * qs.shape[0]
    if workers <= 1 or terms < 4_000_000:
        return _chunk_sum((ys, xs, qs, ps, amps, lam, pitch, z))
    n_chunks = min(ys.shape[0], workers * 4)
    bounds = np.linspace(0, ys.shape[0], n_chunks + 1).astype(np.int64)
    jobs = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    # the point arrays reach the workers through fork, not through pickling
    _SHARED = (ys, xs, qs, ps, amps, lam, pitch, z)
    try:
        with get_context("fork").Pool(workers) as pool:
            parts = pool.map(_shared_chunk, jobs)
    finally:
        _SHARED = None
    return np.concatenate(parts)


def grid_pixels(ny, nx, y0=0, x0=0, h=None, w=None):
    """Row-major pixel coordinates of the window [y0:y0+h, x0:x0+w]."""
    h = ny - y0 if h is None else h
    w = nx - x0 if w is None else w
    yy, xx = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
    return yy.ravel(), xx.ravel()
