"""Reduced-precision storage forms of the directional grid (bit-exact emulation).

The paper does not state a storage precision.  The precision forms keep, per
(bin, voxel), a mean intensity a and a sample count c, derived from the exact
integer sums by one FP32 division, a32 = fl32(S) / fl32(C), and then:

  form  value stored                                   count stored
  fp32  a32                                            fl32(C)
  fp16  q = rne16(fl32(fl32(a32 - 127.5) * fl32(1/127.5)))
        dequantised a' = fl32(fl32(q * 127.5) + 127.5)   rne16(min(fl32(C), 65504))
  bf16  as fp16 with rounding to bfloat16              rne_bf16(fl32(C))
  fp8   per (bin, 8^3 brick) scale s = max(fl32(m / 448), 2^-20) with m the
        largest fl32(|a32 - 127.5|) over its voxels with C > 0;
        q = rne_e4m3(fl32(fl32(a32 - 127.5) / s)),
        a' = fl32(fl32(q * s) + 127.5)                  per-brick scale
                                                       t = fl32(fl32(Cmax) / 448),
                                                       c' = fl32(rne_e4m3(fl32(fl32(C) / t)) * t)

All rounding is round to nearest, ties to even, from the FP32 intermediate.
e4m3 is the OCP "e4m3fn" format (bias 7, no infinities, largest finite 448);
results beyond 448 saturate to 448.  Every function here is written from the
formats' definitions: a value is rounded to the nearest multiple of its
binade's quantum 2^(e - mantissa_bits), with e clamped to the smallest normal
exponent so that subnormals come out right.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32

# (mantissa bits, smallest normal exponent, largest finite value, saturate?)
FORMATS = {
    "bf16": (7, -126, float(np.finfo(np.float32).max), False),
    "fp16": (10, -14, 65504.0, False),
    "e4m3": (3, -6, 448.0, True),
}


def rne(x, fmt: str) -> np.ndarray:
    """Round float32 values to the nearest ``fmt`` value (ties to even); float64 result."""
    mbits, emin, vmax, sat = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    ax = np.abs(x)
    _, ex = np.frexp(ax)                        # ax = m * 2^ex, m in [0.5, 1)
    e = np.maximum(ex - 1, emin)                # binade exponent, subnormals clamped
    quantum = np.ldexp(1.0, e - mbits)
    r = np.rint(ax / quantum) * quantum         # exact scaling; rint ties to even
    r = np.where(ax == 0.0, 0.0, r)
    if sat:
        r = np.minimum(r, vmax)
    else:
        r = np.where(r > vmax, np.inf, r)
    return np.copysign(r, x)


def _f32(x):
    return np.asarray(x, dtype=np.float32)


INV_127_5 = F32(1.0) / F32(127.5)


def mean32(S, C):
    """a32 = fl32(S) / fl32(C) where C > 0, else 0 (float32)."""
    S32, C32 = _f32(S), _f32(C)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = S32 / C32
    return np.where(C32 > 0, a, F32(0.0)).astype(np.float32)


def encode_affine(a32, fmt: str):
    """q for the fp16/bf16 forms (float64 holding the format's value)."""
    x = (_f32(a32) - F32(127.5)).astype(np.float32) * INV_127_5
    return rne(x.astype(np.float32), fmt)


def decode_affine(q) -> np.ndarray:
    return ((_f32(q) * F32(127.5)).astype(np.float32) + F32(127.5)).astype(np.float32)


def brick_reduce_max(x, brick: int = 8):
    """Max over each 8^3 brick of a (K, nz, ny, nx) array (grid padded with -inf)."""
    K, nz, ny, nx = x.shape
    bz, by, bx = -(-nz // brick), -(-ny // brick), -(-nx // brick)
    pad = np.full((K, bz * brick, by * brick, bx * brick), -np.inf)
    pad[:, :nz, :ny, :nx] = x
    return pad.reshape(K, bz, brick, by, brick, bx, brick).max(axis=(2, 4, 6))


def brick_expand(b, shape, brick: int = 8):
    K, nz, ny, nx = shape
    e = np.repeat(np.repeat(np.repeat(b, brick, axis=1), brick, axis=2), brick, axis=3)
    return e[:, :nz, :ny, :nx]


def fp8_scales(S, C, brick: int = 8):
    """Per (bin, brick) FP32 scales (s_value, s_count) of the fp8 form."""
    a32 = mean32(S, C)
    dev = np.abs((a32 - F32(127.5)).astype(np.float32)).astype(np.float64)
    dev = np.where(np.asarray(C) > 0, dev, -np.inf)
    m = brick_reduce_max(dev, brick)
    m = np.where(np.isfinite(m), m, 0.0).astype(np.float32)
    s_val = np.maximum((m / F32(448.0)).astype(np.float32), F32(2.0 ** -20)).astype(np.float32)
    cm = brick_reduce_max(np.where(np.asarray(C) > 0, np.asarray(C, np.float64), -np.inf), brick)
    cm = np.where(np.isfinite(cm), cm, 448.0).astype(np.float32)
    s_cnt = (cm / F32(448.0)).astype(np.float32)
    return s_val, s_cnt


def fp8_encode(S, C, brick: int = 8):
    """Codes and scales of the fp8 form: (q_value, q_count, s_value, s_count).

    q_value, q_count: float64 arrays of e4m3 values, 0 where C == 0;
    s_value, s_count: per (bin, brick) float32 scales from ``fp8_scales``.
    The voxel of a brick farthest from 127.5 encodes to +-448, and so does
    the brick's largest count.
    """
    S = np.asarray(S)
    C = np.asarray(C)
    has = C > 0
    a32 = mean32(S, C)
    s_val, s_cnt = fp8_scales(S, C, brick)
    sv = brick_expand(s_val, S.shape, brick)
    sc = brick_expand(s_cnt, S.shape, brick)
    x = ((a32 - F32(127.5)).astype(np.float32) / sv).astype(np.float32)
    qv = np.where(has, rne(x, "e4m3"), 0.0)
    qc = np.where(has, rne((_f32(C) / sc).astype(np.float32), "e4m3"), 0.0)
    return qv, qc, s_val, s_cnt


def storage(S, C, form: str, brick: int = 8):
    """Dequantised (a', c') float32 arrays exactly as a reader of ``form`` sees them."""
    S = np.asarray(S)
    C = np.asarray(C)
    a32 = mean32(S, C)
    C32 = _f32(C)
    has = C > 0
    if form == "fp32":
        a, c = a32, C32
    elif form in ("fp16", "bf16"):
        fmt = "fp16" if form == "fp16" else "bf16"
        a = decode_affine(encode_affine(a32, fmt))
        cc = np.minimum(C32, F32(65504.0)) if form == "fp16" else C32
        c = rne(cc, fmt).astype(np.float32)
    elif form == "fp8":
        qv, qc, s_val, s_cnt = fp8_encode(S, C, brick)
        sv = brick_expand(s_val, S.shape, brick)
        sc = brick_expand(s_cnt, S.shape, brick)
        a = ((qv.astype(np.float32) * sv).astype(np.float32) + F32(127.5)).astype(np.float32)
        c = (qc.astype(np.float32) * sc).astype(np.float32)
    else:
        raise ValueError(form)
    a = np.where(has, a, F32(0.0)).astype(np.float32)
    c = np.where(has, c, F32(0.0)).astype(np.float32)
    return a, c
