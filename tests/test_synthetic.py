"""The seeded input generator (``synthetic``): Philox4x32-10 against the
published known-answer vectors, the Box-Muller deviates against N(0, 1),
and the shape of the initial field (2/3 box, |k| <= kmax, solenoidal)."""
import numpy as np
import pytest

from synthetic import initial_field, mode_numbers, normal_pairs, philox4x32_10


def _one(ctr, key):
    out = philox4x32_10([np.array([c], dtype=np.uint64) for c in ctr], key)
    return [int(o[0]) for o in out]


@pytest.mark.parametrize("ctr,key,want", [
    # known-answer vectors published with the Philox definition (Salmon et
    # al., SC 2011; the Random123 distribution's kat_vectors)
    ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
    ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
    ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
     [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
])
def test_philox_known_answers(ctr, key, want):
    assert _one(ctr, key) == want


def test_box_muller_deviates_are_standard_normal():
    n = 40000
    kx = np.arange(n) % 401 - 200
    ky = np.arange(n) // 401 - 50
    re, im = normal_pairs(12345, kx, ky, np.zeros(n, dtype=np.int64))
    z = np.concatenate([re, im])
    assert abs(z.mean()) < 4 / np.sqrt(2 * n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / (2 * n))
    # fourth moment 3 and the correlation of re with im near 0
    assert abs(np.mean(z ** 4) - 3.0) < 0.1
    assert abs(np.corrcoef(re, im)[0, 1]) < 0.02


@pytest.mark.parametrize("N,kz,kmax", [(16, 0.57, 4.0), (64, 1.0, 10.0), (32, 0.0, 40.0)])
def test_initial_field_support_and_divergence(N, kz, kmax):
    b = initial_field(N, kz, 99, amp=1.0, kmax=kmax)
    k = mode_numbers(N)
    KX, KY = np.meshgrid(k, k)
    K = (N - 1) // 3
    inside = (np.abs(KX) <= K) & (np.abs(KY) <= K) & (KX ** 2 + KY ** 2 <= kmax ** 2)
    assert np.all(b[:, ~inside] == 0)
    assert np.count_nonzero(b[:, inside]) >= 2 * inside.sum()
    div = KX * b[0] + KY * b[1] + kz * b[2]
    assert np.max(np.abs(div)) <= 1e-14 * np.max(np.abs(b)) * max(K, 1)


def test_initial_field_draw_depends_on_mode_not_grid():
    """A mode's draw is keyed by its wavenumbers, so the same seed gives the
    same coefficients on every grid that holds the mode."""
    a, b = initial_field(32, 0.57, 5), initial_field(128, 0.57, 5)
    k32, k128 = mode_numbers(32).astype(int), mode_numbers(128).astype(int)
    for iy in range(32):
        for ix in range(32):
            if a[0, iy, ix] != 0:
                jy = int(np.nonzero(k128 == k32[iy])[0][0])
                jx = int(np.nonzero(k128 == k32[ix])[0][0])
                assert np.array_equal(a[:, iy, ix], b[:, jy, jx])


@pytest.mark.parametrize("N,kz,seed,amp,kmax", [
    (32, 0.57, 7, 1e-3, 4.0), (128, 1.0, 200000, 1e-3, 4.0), (64, 0.0, 2 ** 63 + 5, 1.0, 20.0),
    (512, 0.57, 500000, 1e-3, 4.0), (16, -2.5, 1, 3.0, 100.0)])
def test_library_generator_is_bitwise_the_same(N, kz, seed, amp, kmax):
    """The C library's host-side generator (pd_seed_field: no device work)
    writes the same bits as this module for the same recipe."""
    import ctypes
    import paper_1902_00387_amd as pd
    out = np.empty((3, N, N), np.complex128)
    st = pd.lib.pd_seed_field(N, kz, ctypes.c_uint64(seed), amp, kmax,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert st == pd.OK
    ref = initial_field(N, kz, seed, amp=amp, kmax=kmax)
    assert np.array_equal(out.view(np.uint64), ref.view(np.uint64))


def test_library_generator_rejects_bad_arguments():
    import ctypes
    import paper_1902_00387_amd as pd
    out = np.empty((3, 48, 48), np.complex128)
    p = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert pd.lib.pd_seed_field(48, 0.5, 1, 1.0, 4.0, p) == pd.EINVAL
    assert pd.lib.pd_seed_field(32, float("nan"), 1, 1.0, 4.0, p) == pd.EINVAL
    assert pd.lib.pd_seed_field(32, 0.5, 1, 1.0, 4.0, None) == pd.EINVAL
