"""Oracle FFT: iterative radix-2 Cooley-Tukey, plus a brute-force DFT.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The FS scheme (Sec. 2.2, Algorithm 1) applies the discrete Fourier
transform F and its inverse to whole fields every step.  The paper leaves
the normalisation unstated; the scheme is invariant to it.  This module
uses the plain definitions

    forward  X[k] = sum_j x[j] exp(-2 pi i j k / N)       (unnormalised)
    inverse  x[j] = (1/N) sum_k X[k] exp(+2 pi i j k / N)

applied axis by axis for multi-dimensional arrays.  Lengths must be powers
of two for `fft_axis`; `dft_brute` accepts any length and is the O(N^2)
textbook sum used to pin `fft_axis`.
"""

import numpy as np


def _is_pow2(n):
    return n >= 1 and (n & (n - 1)) == 0


def _bit_reverse_indices(n):
    bits = n.bit_length() - 1
    idx = np.arange(n, dtype=np.int64)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


def fft_axis(a, axis=-1, inverse=False):
    """Radix-2 decimation-in-time FFT of `a` along `axis` (complex128).

    The input is permuted into bit-reversed order, then log2(N) butterfly
    stages combine pairs of half-length transforms:
        X[k]       = E[k] + w^k O[k]
        X[k + m/2] = E[k] - w^k O[k],   w = exp(-+2 pi i / m).
    The inverse uses the conjugate twiddles and divides by N.
    """
    x = np.moveaxis(np.asarray(a, dtype=np.complex128), axis, -1)
    lead = x.shape[:-1]
    n = x.shape[-1]
    if not _is_pow2(n):
        raise ValueError("fft_axis needs a power-of-two length, got %d" % n)
    x = x[..., _bit_reverse_indices(n)]
    sign = 1.0 if inverse else -1.0
    m = 2
    while m <= n:
        half = m // 2
        w = np.exp(sign * 2j * np.pi * np.arange(half) / m)
        blocks = x.reshape(lead + (n // m, m))
        even = blocks[..., :half]
        odd = blocks[..., half:] * w
        x = np.concatenate([even + odd, even - odd], axis=-1).reshape(lead + (n,))
        m *= 2
    if inverse:
        x = x / n
    return np.moveaxis(x, -1, axis)


def _per_slice(a, axes, inverse, workers):
    """Transform each slice a[f] along the leading axis (which is not in
    `axes`) in its own task on `workers` threads.  Every slice goes through
    exactly the operations it would get as part of the batch, so the result
    is bit-identical to the serial call; NumPy releases the interpreter lock
    inside its array operations, so large slices run in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    a = np.asarray(a, dtype=np.complex128)
    sub = tuple(ax - 1 for ax in axes)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(lambda f: _transform(a[f], sub, inverse), range(a.shape[0])))
    return np.stack(parts)


def _transform(a, axes, inverse):
    out = np.asarray(a, dtype=np.complex128)
    for ax in axes:
        out = fft_axis(out, ax, inverse=inverse)
    return out


def fftn(a, axes, workers=1):
    """Forward transform over every axis in `axes` (unnormalised).

    `workers` > 1 transforms the slices along a leading axis that is not in
    `axes` (the fields) on that many threads, with a bit-identical result."""
    if workers > 1 and np.ndim(a) > 1 and 0 not in axes:
        return _per_slice(a, axes, False, workers)
    return _transform(a, axes, False)


def ifftn(a, axes, workers=1):
    """Inverse transform over every axis in `axes` (normalised by 1/N per
    axis); `workers` as for `fftn`."""
    if workers > 1 and np.ndim(a) > 1 and 0 not in axes:
        return _per_slice(a, axes, True, workers)
    return _transform(a, axes, True)


def dft_brute(a, axes, inverse=False):
    """Textbook O(N^2) DFT along each axis: an explicit sum over j for each k.

    Used only to pin `fft_axis`.  Any length.
    """
    out = np.asarray(a, dtype=np.complex128)
    sign = 1.0 if inverse else -1.0
    for ax in axes:
        n = out.shape[ax]
        j = np.arange(n)
        mat = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        if inverse:
            mat = mat / n
        moved = np.moveaxis(out, ax, -1)
        res = np.zeros_like(moved)
        for k in range(n):
            acc = np.zeros(moved.shape[:-1], dtype=np.complex128)
            for jj in range(n):
                acc = acc + moved[..., jj] * mat[k, jj]
            res[..., k] = acc
        out = np.moveaxis(res, -1, ax)
    return out
