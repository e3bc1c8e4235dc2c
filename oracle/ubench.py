"""What the measurement kernels compute, written out plainly (numpy, FP64) —
TEST INFRASTRUCTURE ONLY.

The microbenchmarks of the paper's calibration set (Section "Measurement
Kernel Design") each exercise one operation; their outputs are defined so that
a test can confirm the kernel did the work it is timed for:
  stream    the elementwise sum of the inputs;
  strided   a gather at stride S;
  fma       32 registers r_v = (t mod 256) / 2^8 + v / 2^5 per thread t, each
            loop trip applying r_v <- -r_v / 2 + r_{(v+16) mod 32} for v = 0..31
            and then again (64 updates), the registers' sum stored;
  mfma      eight accumulators of `iters` 16x16 matrix products each, operand
            values a(l) = (3l mod 7) - 3 and b(l) = (5l mod 9) - 4 supplied by lane l
            to every position it holds;
  lds       every wave's 64 values rotated by `iters` lanes;
  barrier   the barrier count;
  overlap   every wave's 64 vectors rotated by m lanes (zeros past the end);
  tile_read out[i][j] = sum over k < n/16 of x[i][16k + j mod 16] (pattern a)
            or of x[16k + i mod 16][j] (pattern b).
Inputs of the tests are small integers or dyadic fractions, so FP64 here and
FP32 on the GPU agree exactly.
"""
from __future__ import annotations

import numpy as np


def stream(inputs):
    out = np.zeros_like(np.asarray(inputs[0], dtype=np.float64))
    for x in inputs:
        out = out + np.asarray(x, dtype=np.float64)
    return out


def strided(x, n, S):
    return np.asarray(x, dtype=np.float64)[np.arange(n) * S]


def fma(nwg, iters):
    t = np.arange(256 * nwg) % 256
    r = [t * 2.0 ** -8 + v * 2.0 ** -5 for v in range(32)]
    for _ in range(iters):
        for k in range(64):
            v = k % 32
            r[v] = -0.5 * r[v] + r[(v + 16) % 32]
    s = r[0].copy()
    for v in range(1, 32):
        s = s + r[v]
    return s


def _mfma_wave(dtype):
    """One wave's 16x16 product in the matrix cores' register layout: lane l
    of the 16x16 result holds rows 4(l // 16) .. +3 of column l % 16.  FP32
    16x16x4: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k.  BF16
    16x16x32: lane i + 16g holds eight A entries of row i (all a(i + 16g)),
    lane j + 16g eight B entries of column j, their k ranges disjoint."""
    lanes = np.arange(64)
    a = ((3 * lanes) % 7 - 3).astype(np.float64)
    b = ((5 * lanes) % 9 - 4).astype(np.float64)
    rep = 8 if dtype == "bf16" else 1
    D = np.zeros((16, 16))
    for i in range(16):
        for j in range(16):
            D[i, j] = sum(rep * a[i + 16 * g] * b[j + 16 * g] for g in range(4))
    out = np.zeros((64, 4))
    for l in range(64):
        for r in range(4):
            out[l, r] = D[4 * (l // 16) + r, l % 16]
    return out


def mfma(nwg, iters, dtype="f32"):
    w = 8 * iters * _mfma_wave(dtype)
    return np.tile(w.reshape(-1), 4 * nwg)


def lds(x, nwg, iters, width):
    x = np.asarray(x, dtype=np.float64).reshape(4 * nwg, 64, width)
    return np.roll(x, -iters, axis=1).reshape(-1)


def barrier(nwg, iters):
    return np.full(256 * nwg, float(iters))


def overlap(x, n4, m):
    x = np.asarray(x, dtype=np.float64).reshape(n4, 4)
    blocks = -(-n4 // 256)
    pad = np.zeros((256 * blocks, 4))
    pad[:n4] = x
    rot = np.roll(pad.reshape(4 * blocks, 64, 4), -m, axis=1).reshape(-1, 4)
    return rot[:n4].reshape(-1)


def tile_read(x, n, pattern):
    x = np.asarray(x, dtype=np.float64).reshape(n, n)
    out = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if pattern == 0:
                out[i, j] = sum(x[i, 16 * k + j % 16] for k in range(n // 16))
            else:
                out[i, j] = sum(x[16 * k + i % 16, j] for k in range(n // 16))
    return out.reshape(-1)
