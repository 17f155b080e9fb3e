"""CPU check of the recurrence the Laplacian-input path uses for its float64 low-bin row sums
(k_lap_rows): lane j of a 64-lane wavefront takes the elements x = j + 64 k of a row, runs
Goertzel's second-order recurrence s_k = v_k + 2 Re(z) s_(k-1) - s_(k-2) with z = w^(64 l)
over them (zeros past the row, in chunks of 8 per lane), and closes with s_(n-1) - z s_(n-2)
times the table entry w^(l j + 64 l (n-1)). The lanes' parts must add up to the direct sum
sum_x v_x w^(l x), w = exp(-2 pi i / N), to float64 rounding, including bins where z is real
(64 l a multiple of N / 2)."""
import numpy as np
import pytest


def _lane_sums(v, N, l, chunk=8):
    W1 = len(v)
    m = np.arange(N)
    twr, twi = np.cos(2 * np.pi * m / N), -np.sin(2 * np.pi * m / N)
    iters = 0
    while iters * 64 * chunk <= W1 - 1:
        iters += 1
    n = iters * chunk
    d = (l * 64) % N
    c2, zr, zi = 2 * twr[d], twr[d], twi[d]
    total = 0j
    for lane in range(64):
        s1 = s2 = 0.0
        for k in range(n):
            x = lane + 64 * k
            s0 = c2 * s1 + ((v[x] if x < W1 else 0.0) - s2)
            s2, s1 = s1, s0
        qr, qi = s1 - zr * s2, -zi * s2
        e = (l * lane + l * 64 * (n - 1)) % N
        pr, pi = twr[e], twi[e]
        total += complex(pr * qr - pi * qi, pr * qi + pi * qr)
    return total


@pytest.mark.parametrize("W1,N", [(1201, 2400), (64, 128), (33, 72), (700, 1400), (1, 16),
                                  (129, 256), (1025, 2048)])
def test_lane_goertzel_matches_direct_sum(W1, N):
    rng = np.random.default_rng(W1 + N)
    v = rng.normal(size=W1).astype(np.float32).astype(np.float64)
    for l in range(5):
        direct = np.sum(v * np.exp(-2j * np.pi * l * np.arange(W1) / N))
        got = _lane_sums(v, N, l)
        assert abs(got - direct) <= 1e-12 * max(1.0, np.abs(v).sum()), (W1, N, l, got, direct)
