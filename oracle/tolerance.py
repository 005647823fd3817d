"""Stated accuracy bars of the GPU path against this oracle (test
infrastructure only).

A result passes when its relative Frobenius error against the FP64 oracle is
at most max(ABS, FACTOR * floor), where floor is the oracle's own relative
change when every input entry moves by a random relative +-2^-24 (the
problem's sensitivity to float32-sized input noise; floor_estimate).  At
large p the power is ill-conditioned and no float32 method can reach the
absolute bar; the floor term then takes over.

  float32 products, FP16 hi/lo (3 products) and
  BF16 three parts (6 products):                 ABS 1e-5,  FACTOR 64
  BF16 hi/lo (3 products, about 16 bits each):  ABS 2e-4,  FACTOR 1024
"""
FP32_ABS_TOL = 1e-5
FP32_FLOOR_FACTOR = 64.0
BF16X3_ABS_TOL = 2e-4
BF16X3_FLOOR_FACTOR = 1024.0

# product modes, as numbered by the library's C interface
MODE_FP32, MODE_FP16X3, MODE_BF16X3, MODE_BF16X6 = 0, 1, 2, 3


def tol_fp32(floor: float) -> float:
    return max(FP32_ABS_TOL, FP32_FLOOR_FACTOR * floor)


def tol_mode(mode: int, floor: float) -> float:
    """Stated tolerance per product mode (FP16X3 and BF16X6 share the float32
    bound)."""
    if mode == MODE_BF16X3:
        return max(BF16X3_ABS_TOL, BF16X3_FLOOR_FACTOR * floor)
    return tol_fp32(floor)


def tol_expm(floor: float, squarings: int) -> float:
    """Bar of the float32 matrix exponential (scaling and squaring): the
    float32 bar, or 4 * 2^j * 2^-24 when larger.  The Taylor polynomial of
    B = A 2^-j carries a relative error of a few units of float32 rounding,
    and each of the j squarings doubles a relative error, so the method's own
    error grows as 2^j * 2^-24 whatever the input's sensitivity."""
    return max(tol_fp32(floor), 4.0 * 2.0 ** squarings * 2.0 ** -24)

