"""SplitMix64 and the index draw of the sparse embedding matrix (oracle side).

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014; public-domain reference code by S. Vigna): the state advances by the
odd constant 0x9E3779B97F4A7C15 and each output is the state passed through the
finalizer  z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27; z *= 0x94D049BB133111EB;
z ^= z>>31.  The stream is therefore counter-based: output number a (a >= 1) of the
stream started at state x0 is  fmix(x0 + a * 0x9E3779B97F4A7C15)  modulo 2^64.

Definition 2.1 asks for gamma distinct rows per column, chosen uniformly without
replacement, with independent signs. The paper fixes no generator; the reading used on
both sides of the parity check is:

  * column key      k_i   = output number (i+1) of the stream started at ``seed``;
  * draw a (a>=0)   u     = output number (a+1) of the stream started at k_i;
  * candidate row   floor(hi32(u) * s / 2^32)   (Lemire's multiply-shift reduction);
  * sign            -1 if bit 0 of u is set, else +1;
  * the first gamma distinct candidates in draw order are kept (rejection of repeats).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def fmix64(z: int) -> int:
    """The SplitMix64 output finalizer on a Python int."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_outputs(seed: int, count: int) -> list[int]:
    """The first ``count`` outputs of the SplitMix64 stream seeded with ``seed``,
    stepping the state exactly as the published generator does."""
    x = seed & MASK64
    out = []
    for _ in range(count):
        x = (x + GOLDEN) & MASK64
        out.append(fmix64(x))
    return out


def stream_output(state: int, index: int) -> int:
    """Output number ``index`` (1-based) of the stream started at ``state``."""
    return fmix64((state + index * GOLDEN) & MASK64)


# -- vectorised forms over many columns (numpy uint64 arithmetic wraps mod 2^64) -----
_G = np.uint64(GOLDEN)
_U1 = np.uint64(_M1)
_U2 = np.uint64(_M2)


def _fmix_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _U1
    z = (z ^ (z >> np.uint64(27))) * _U2
    return z ^ (z >> np.uint64(31))


def _stream_output_np(state: np.ndarray, index: int) -> np.ndarray:
    return _fmix_np(state + np.uint64(index) * _G)


def sketch_indices(seed: int, n: int, s: int, gamma: int):
    """Rows (int32, n x gamma) and signs (int8, n x gamma) of a sparse embedding
    matrix S in R^{s x n} (Definition 2.1): column i of S holds sign/sqrt(gamma) at
    rows[i, g] for g < gamma, in draw order."""
    if not (1 <= gamma <= s):
        raise ValueError("need 1 <= gamma <= s")
    with np.errstate(over="ignore"):
        cols = np.arange(n, dtype=np.uint64)
        keys = _fmix_np(np.uint64(seed & MASK64) + (cols + np.uint64(1)) * _G)
        rows = np.full((n, gamma), -1, dtype=np.int64)
        signs = np.zeros((n, gamma), dtype=np.int8)
        count = np.zeros(n, dtype=np.int64)
        a = 0
        while (count < gamma).any():
            a += 1
            todo = np.nonzero(count < gamma)[0]
            u = _stream_output_np(keys[todo], a)
            cand = ((u >> np.uint64(32)) * np.uint64(s)) >> np.uint64(32)
            cand = cand.astype(np.int64)
            sg = np.where((u & np.uint64(1)) == np.uint64(1), -1, 1).astype(np.int8)
            dup = (rows[todo] == cand[:, None]).any(axis=1)
            take = todo[~dup]
            rows[take, count[take]] = cand[~dup]
            signs[take, count[take]] = sg[~dup]
            count[take] += 1
    return rows.astype(np.int32), signs


def sketch_indices_loop(seed: int, n: int, s: int, gamma: int):
    """The same draw written as a plain per-column loop on Python ints (slow; used to
    pin the vectorised form on small sizes)."""
    rows = np.zeros((n, gamma), dtype=np.int32)
    signs = np.zeros((n, gamma), dtype=np.int8)
    for i in range(n):
        key = stream_output(seed, i + 1)
        got, a = [], 0
        while len(got) < gamma:
            a += 1
            u = stream_output(key, a)
            r = ((u >> 32) * s) >> 32
            if any(r == g[0] for g in got):
                continue
            got.append((r, -1 if (u & 1) else 1))
        rows[i] = [g[0] for g in got]
        signs[i] = [g[1] for g in got]
    return rows, signs


# -- Gaussian probes (Hutchinson's estimator of Section 3.2 draws them; the paper fixes
# no generator). Box and Muller (1958) over the same counter-based stream:
#   probe key        k_j = output number (j+1) of the stream started at seed ^ PROBE_DOMAIN;
#   element i        u1 = output (2i+1), u2 = output (2i+2) of the stream started at k_j;
#                    U1 = (hi53(u1) + 1) 2^-53 in (0, 1],  U2 = hi53(u2) 2^-53 in [0, 1);
#                    g = sqrt(-2 ln U1) cos(2 pi U2).
# The domain constant keeps a probe block and a sketch drawn from the same seed apart.
PROBE_DOMAIN = 0xD1B54A32D192ED03


def probe_uniforms(seed: int, n: int, N: int):
    """(U1, U2), each (N, n) float64, of the probe generator."""
    with np.errstate(over="ignore"):
        j = np.arange(N, dtype=np.uint64)[:, None]
        i = np.arange(n, dtype=np.uint64)[None, :]
        keys = _fmix_np(np.uint64((seed ^ PROBE_DOMAIN) & MASK64) + (j + np.uint64(1)) * _G)
        u1 = _fmix_np(keys + (np.uint64(2) * i + np.uint64(1)) * _G)
        u2 = _fmix_np(keys + (np.uint64(2) * i + np.uint64(2)) * _G)
    U1 = ((u1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    U2 = (u2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return U1, U2


def gaussian_probes(seed: int, n: int, N: int) -> np.ndarray:
    """N probes of length n, (N, n) float64, by Box-Muller on probe_uniforms."""
    U1, U2 = probe_uniforms(seed, n, N)
    return np.sqrt(-2.0 * np.log(U1)) * np.cos(2.0 * np.pi * U2)
