"""XTS-AES on the GPU against the oracle's XTS, bit for bit, through the C ABI.

Small and ragged buffers (several groups of 64 data units, a last unit
shorter than the others, a last group that is not full) are compared whole;
the 1 GiB buffer the benchmark times is compared on sampled data units that
the oracle encrypts one by one with their own tweak value, plus
decrypt(encrypt(x)) == x over the whole buffer.
"""
import numpy as np
import pytest

import seedgen
from oracle import ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def A():
    from paper_1403_7295_amd import aesgpu
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return aesgpu


@pytest.fixture(scope="module")
def O():
    return ref.default()


def keys(A, master, index, bits):
    rk1, nr = A.aes_expand_key(seedgen.key(master, 2 * index, bits))
    rk2, _ = A.aes_expand_key(seedgen.key(master, 2 * index + 1, bits))
    return rk1, rk2, nr


def gpu_xts(A, decrypt, x_np, rk1, rk2, nr, unit, first, inplace=False):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to("cuda")
    out = x if inplace else torch.empty_like(x)
    fn = A.aes_xts_decrypt if decrypt else A.aes_xts_encrypt
    fn(x, out, x_np.size, rk1, rk2, nr, unit, first)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError("%s: %d bytes differ, first at %d (block %d)"
                             % (what, bad.size, bad[0], bad[0] // 16))


# (unit bytes, buffer bytes): several 64-unit groups, ragged last unit and group
CASES = [
    (16, 16), (16, 64 * 16 * 3 + 48),
    (32, 32 * 200 + 16),
    (64, 64 * 130),
    (512, 512 * 64 * 2 + 512 * 5 + 240),
    (1024, 1024 * 70 + 1008),
    (4096, 4096 * 64 + 4096 * 3 + 2064),
    (4096, 16),
]


@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("unit,nbytes", CASES, ids=["u%d-n%d" % c for c in CASES])
def test_xts_matches_oracle(A, O, bits, unit, nbytes):
    rk1, rk2, nr = keys(A, 40, unit, bits)
    first = 1000 + unit
    x = seedgen.data_np(40, bits + unit, nbytes)
    what = "XTS-AES-%d unit %d, %d bytes" % (bits, unit, nbytes)
    ct = gpu_xts(A, False, x, rk1, rk2, nr, unit, first)
    assert_same(ct, O.xts(False, rk1, rk2, nr, unit, first, x), what + " encrypt")
    # decryption on its own (random input), and the round trip
    assert_same(gpu_xts(A, True, x, rk1, rk2, nr, unit, first),
                O.xts(True, rk1, rk2, nr, unit, first, x), what + " decrypt")
    assert_same(gpu_xts(A, True, ct, rk1, rk2, nr, unit, first), x, what + " round trip")


@pytest.mark.parametrize("first", [0, (1 << 32) - 3, (1 << 64) - 70])
def test_xts_tweak_values(A, O, first):
    # tweak values across 2^32 (a carry into the second word) and across 2^64
    # (the unit number wraps modulo 2^64 on both sides)
    rk1, rk2, nr = keys(A, 41, 0, 256)
    x = seedgen.data_np(41, 1, 512 * 140)
    assert_same(gpu_xts(A, False, x, rk1, rk2, nr, 512, first),
                O.xts(False, rk1, rk2, nr, 512, first, x), "first unit %d" % first)


@pytest.mark.parametrize("decrypt", [False, True])
def test_xts_in_place(A, O, decrypt):
    rk1, rk2, nr = keys(A, 42, 0, 128)
    x = seedgen.data_np(42, 1, 4096 * 70 + 512)
    assert_same(gpu_xts(A, decrypt, x, rk1, rk2, nr, 4096, 7, inplace=True),
                O.xts(decrypt, rk1, rk2, nr, 4096, 7, x), "in place")


def test_xts_same_keys_is_still_defined(A, O):
    # K1 == K2 is outside what the standard recommends, but the operation is
    # well defined and both sides compute it the same way
    rk1, _, nr = keys(A, 43, 0, 128)
    x = seedgen.data_np(43, 1, 512 * 66)
    assert_same(gpu_xts(A, False, x, rk1, rk1, nr, 512, 5),
                O.xts(False, rk1, rk1, nr, 512, 5, x), "K1 == K2")


@pytest.mark.parametrize("bits,unit", [(128, 4096), (256, 512)])
def test_xts_1gib_sampled(A, O, bits, unit):
    n = 1 << 30
    master = 44
    rk1, rk2, nr = keys(A, master, 0, bits)
    first = 123456789
    x = seedgen.data_torch(master, bits, n, "cuda")
    y = torch.empty_like(x)
    A.aes_xts_encrypt(x, y, n, rk1, rk2, nr, unit, first)
    torch.cuda.synchronize()
    nunits = n // unit
    rng = np.random.default_rng(unit)
    units = np.unique(np.concatenate([rng.integers(0, nunits, 48), [0, 63, 64, nunits - 1]]))
    yv = y.view(-1, unit)
    for u in units:
        u = int(u)
        xu = seedgen.data_np(master, bits, unit, offset=unit * u)
        want = O.xts(False, rk1, rk2, nr, unit, first + u, xu)
        assert_same(yv[u].cpu().numpy(), want, "1 GiB unit %d" % u)
    z = torch.empty_like(x)
    A.aes_xts_decrypt(y, z, n, rk1, rk2, nr, unit, first)
    torch.cuda.synchronize()
    assert torch.equal(z, x), "decrypt(encrypt(x)) != x over 1 GiB"
    del x, y, z
    torch.cuda.empty_cache()
