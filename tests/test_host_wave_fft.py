"""Host model of the in-wave 1024-point transform of the pass kernels (csrc/wave_fft.hpp).

The kernel factors 1024 = 4 x 256: a radix-4 in registers, one exchange between the four
waves, then a 256-point transform inside each wave whose lane digits are brought into the
register slots by cross-lane exchanges (permlane swaps for lane bits 5:4, bank-masked DPP row
shifts for bits 3:2, the wave's own LDS quarter for bits 1:0).  This test replays those steps
on arrays of [wave][lane][slot] with the documented semantics of each cross-lane operation
and checks the result against numpy's FFT in the bin order the kernel assumes (wave_bin),
the inverse against the identity, and the filter between them against a circular
convolution; the GPU lane-layout of the same operations is covered by the parity tests.
"""
import numpy as np

LANE = np.arange(64)


def dft4(a, inv):
    s = 1 if inv else -1
    m = np.exp(s * 2j * np.pi * np.outer(np.arange(4), np.arange(4)) / 4)
    return a @ m.T


def permlane32_swap(lo, hi):
    # lanes 32..63 of lo <-> lanes 0..31 of hi
    lo2, hi2 = lo.copy(), hi.copy()
    lo2[32:], hi2[:32] = hi[:32], lo[32:]
    return lo2, hi2


def permlane16_swap(lo, hi):
    # odd 16-lane rows of lo <-> even rows of hi
    lo2, hi2 = lo.copy(), hi.copy()
    for r in (0, 2):
        lo2[(r + 1) * 16:(r + 2) * 16] = hi[r * 16:(r + 1) * 16]
        hi2[r * 16:(r + 1) * 16] = lo[(r + 1) * 16:(r + 2) * 16]
    return lo2, hi2


def update_dpp_row(old, src, shr, d, bank_mask):
    # row_shr:d reads lane i - d, row_shl:d lane i + d, inside 16-lane rows; lanes outside
    # the bank mask (banks = groups of 4 lanes of a row) or with an out-of-row source keep old
    out = old.copy()
    for i in range(64):
        if not (bank_mask >> ((i >> 2) & 3)) & 1:
            continue
        j = i - d if shr else i + d
        if j // 16 == i // 16:
            out[i] = src[j]
    return out


def swap_row(lo, hi, d):
    bm_set, bm_clear = (0xC, 0x3) if d == 8 else (0xA, 0x5)
    return update_dpp_row(lo, hi, True, d, bm_set), update_dpp_row(hi, lo, False, d, bm_clear)


def transpose_low(a):
    # the LDS exchange of lane bits 1:0 with the slot, with the kernel's rotated addresses
    own = np.zeros(256, complex)
    for j in range(4):
        own[64 * j + ((LANE + j) & 63)] = a[:, j]
    d = LANE & 3
    src = LANE & ~3
    return np.stack([own[64 * d + ((src + j + d) & 63)] for j in range(4)], 1)


def transpose(a, sh):
    a = a.copy()
    if sh == 4:
        for i, j in ((0, 2), (1, 3)):
            a[:, i], a[:, j] = permlane32_swap(a[:, i], a[:, j])
        for i, j in ((0, 1), (2, 3)):
            a[:, i], a[:, j] = permlane16_swap(a[:, i], a[:, j])
    elif sh == 2:
        for i, j in ((0, 2), (1, 3)):
            a[:, i], a[:, j] = swap_row(a[:, i], a[:, j], 8)
        for i, j in ((0, 1), (2, 3)):
            a[:, i], a[:, j] = swap_row(a[:, i], a[:, j], 4)
    else:
        a = transpose_low(a)
    return a


T = np.arange(256)
L = T & 63
TW = np.exp(-2j * np.pi * np.arange(1024) / 1024)
TWR = np.zeros((256, 12), complex)
for _j in (1, 2, 3):
    TWR[:, _j - 1] = TW[(T * _j) & 1023]
    TWR[:, 2 + _j] = TW[4 * L * _j]
    TWR[:, 5 + _j] = TW[16 * (L & 15) * _j]
    TWR[:, 8 + _j] = TW[64 * (L & 3) * _j]


def twiddle(a, o, inv, tws):
    a = a.copy()
    for j in (1, 2, 3):
        a[:, j] *= np.conj(tws[:, o + j - 1]) if inv else tws[:, o + j - 1]
    return a


def forward(x):
    v = np.stack([x[T + 256 * q] for q in range(4)], 1)
    v = twiddle(dft4(v, False), 0, False, TWR)
    buf = np.zeros(1024, complex)
    for k in range(4):
        buf[k * 256 + T] = v[:, k]
    v = np.stack([buf[(T >> 6) * 256 + L + 64 * r] for r in range(4)], 1)
    out = np.zeros_like(v)
    for w in range(4):
        a, tws = v[w * 64:(w + 1) * 64], TWR[w * 64:(w + 1) * 64]
        a = twiddle(dft4(a, False), 3, False, tws)
        a = twiddle(dft4(transpose(a, 4), False), 6, False, tws)
        a = twiddle(dft4(transpose(a, 2), False), 9, False, tws)
        out[w * 64:(w + 1) * 64] = dft4(transpose(a, 0), False)
    return out


def inverse(v):
    out = np.zeros_like(v)
    for w in range(4):
        a, tws = v[w * 64:(w + 1) * 64], TWR[w * 64:(w + 1) * 64]
        a = dft4(twiddle(transpose(dft4(a, True), 0), 9, True, tws), True)
        a = dft4(twiddle(transpose(a, 2), 6, True, tws), True)
        a = dft4(twiddle(transpose(a, 4), 3, True, tws), True)
        out[w * 64:(w + 1) * 64] = a
    buf = np.zeros(1024, complex)
    for r in range(4):
        buf[(T >> 6) * 256 + L + 64 * r] = out[:, r]
    v = np.stack([buf[k * 256 + T] for k in range(4)], 1)
    v = dft4(twiddle(v, 0, True, TWR), True)
    x = np.zeros(1024, complex)
    for q in range(4):
        x[T + 256 * q] = v[:, q]
    return x


def wave_bin(t, q):
    return (t >> 6) + 4 * ((t >> 4) & 3) + 16 * ((t >> 2) & 3) + 64 * (t & 3) + 256 * q


BINS = np.array([[wave_bin(t, q) for q in range(4)] for t in range(256)])


def test_bins_are_a_permutation():
    assert sorted(BINS.ravel().tolist()) == list(range(1024))


def test_slot_lane_exchanges_are_involutions_of_the_digit():
    a = (np.arange(64)[:, None] * 4 + np.arange(4)[None, :]).astype(complex)   # value = 4 lane + slot
    for sh in (4, 2, 0):
        b = transpose(a, sh)
        d = (LANE >> sh) & 3
        for j in range(4):
            src_lane = (LANE & ~(3 << sh)) | (j << sh)
            assert np.array_equal(b[:, j], a[src_lane, d])
        assert np.array_equal(transpose(b, sh), a)


def test_forward_is_the_dft_in_wave_bin_order():
    r = np.random.default_rng(1)
    x = r.standard_normal(1024) + 1j * r.standard_normal(1024)
    X = np.fft.fft(x)
    assert np.max(np.abs(forward(x) - X[BINS])) <= 1e-12 * np.max(np.abs(X))


def test_inverse_of_forward_and_the_filter_between_them():
    r = np.random.default_rng(2)
    x = r.standard_normal(1024) + 1j * r.standard_normal(1024)
    assert np.max(np.abs(inverse(forward(x)) / 1024 - x)) <= 1e-12
    h = np.exp(1j * r.standard_normal(1024))
    y = inverse(forward(x) * h[BINS]) / 1024
    assert np.max(np.abs(y - np.fft.ifft(np.fft.fft(x) * h))) <= 1e-12
