"""The high-multiply division the network kernels use for pixel rows and
columns (SmallDiv in csrc/fwi_nn.hip): floor(n / d) = (n m) >> 32 with
m = floor((2^32 - 1) / d) + 1, claimed exact for n d < 2^32.  Checked here
in exact integer arithmetic over every divisor the kernels can see
(1 <= d <= 2^15; d = 1 is passed through) at the ends of the range they use
(n < 2 d + 2^9: a column or row index plus at most a block of
pixels) and at every multiple of d and its neighbours below that,
plus random n with n d < 2^32."""
import numpy as np


def _smalldiv(n, d):
    if d <= 1:
        return n
    m = ((1 << 32) - 1) // d + 1
    return (n * m) >> 32


def test_exact_on_the_kernels_range():
    for d in range(1, 32769):
        top = 2 * d + 512
        ns = {0, 1, top - 1, top - 2}
        for k in range(1, top // d + 1):
            ns.update((k * d - 1, k * d, k * d + 1))
        for n in ns:
            if 0 <= n < top:
                assert _smalldiv(n, d) == n // d, (n, d)


def test_exact_wherever_n_d_below_2_32():
    rng = np.random.default_rng(7)
    for d in list(range(2, 300)) + [int(v) for v in rng.integers(300, 1 << 16, 2000)]:
        limit = ((1 << 32) - 1) // d
        for n in [limit, limit - 1] + [int(v) for v in rng.integers(0, limit + 1, 20)]:
            assert _smalldiv(n, d) == n // d, (n, d)
