"""AES-GCM on the GPU against the oracle's GCM, bit for bit (ciphertext and
tag), through the C ABI.

Small and ragged cases are compared whole: empty plaintexts (GMAC), partial
last blocks, additional data of any length, IVs of 12 and of other lengths,
buffers that use one workgroup and buffers that use all 256 (16 MiB).  The
1 GiB buffer the benchmark times is checked on sampled ciphertext blocks
(oracle CTR from J0 + 1) and on the tag through GHASH's linearity: changing
plaintext block j by d changes the tag by d * H^(nC - j + 1), a product the
oracle computes directly.
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


@pytest.fixture(scope="module")
def ws(A):
    return torch.zeros(A.aes_gcm_workspace_size(), dtype=torch.uint8, device="cuda")


def dev(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    t = torch.empty(max(a.size, 16), dtype=torch.uint8, device="cuda")
    if a.size:
        t[:a.size] = torch.from_numpy(a).to("cuda")
    return t


def gpu_encrypt(A, ws, rk, nr, iv, aad, pt):
    x, ad = dev(pt), dev(aad)
    y = torch.empty_like(x)
    tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
    A.aes_gcm_encrypt(x, y, pt.size, ad, aad.size, rk, nr, iv, tag, ws)
    torch.cuda.synchronize()
    return y[:pt.size].cpu().numpy(), tag.cpu().numpy()


def gpu_decrypt(A, ws, rk, nr, iv, aad, ct, tag):
    x, ad = dev(ct), dev(aad)
    y = torch.empty_like(x)
    t = dev(tag)
    ok = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    A.aes_gcm_decrypt(x, y, ct.size, ad, aad.size, rk, nr, iv, t, tag.size, ok, ws)
    torch.cuda.synchronize()
    return y[:ct.size].cpu().numpy(), int(ok.item())


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError("%s: %d bytes differ, first at %d" % (what, bad.size, bad[0]))


CASES = [(0, 0), (0, 45), (1, 0), (15, 16), (16, 0), (17, 33), (4096, 20), (65536 + 7, 1000),
         ((1 << 20) + 33, 17), (3 * (1 << 20) + 5, 4096 * 16 + 3)]


@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("nbytes,aad_bytes", CASES, ids=["p%d-a%d" % c for c in CASES])
def test_gcm_matches_oracle(A, O, ws, bits, nbytes, aad_bytes):
    rk, nr = A.aes_expand_key(seedgen.key(50, nbytes % 1000, bits))
    iv = seedgen.nonce(50, bits)[:12]
    pt = seedgen.data_np(50, nbytes, nbytes)
    aad = seedgen.data_np(51, aad_bytes, aad_bytes)
    want_ct, want_tag = O.gcm_encrypt(rk, nr, iv, aad, pt)
    ct, tag = gpu_encrypt(A, ws, rk, nr, iv, aad, pt)
    what = "GCM-%d, %d B plaintext, %d B AAD" % (bits, nbytes, aad_bytes)
    assert_same(ct, want_ct, what + " ciphertext")
    assert_same(tag, want_tag, what + " tag")
    back, ok = gpu_decrypt(A, ws, rk, nr, iv, aad, ct, tag)
    assert ok == 1, what + ": own tag rejected"
    assert_same(back, pt, what + " decrypt")


def test_gcm_every_head_length(A, O, ws):
    """The last (nC + 1) mod 64 hash positions (the length block and the
    ragged end of the ciphertext) are finished apart from the bulk, so that
    the bulk's slots start on 1 KiB boundaries: every such count 0 .. 63,
    with and without a partial last block, in both directions, and once
    with enough blocks for several chunks per wave."""
    rk, nr = A.aes_expand_key(seedgen.key(59, 0, 128))
    iv = seedgen.nonce(59, 0)[:12]
    aad = seedgen.data_np(59, 1, 37)
    heads = set()
    for nblk in list(range(700, 764)) + [(1 << 16) + 5, (1 << 16) + 62]:
        for tail in (0, 9):
            nbytes = 16 * nblk - (16 - tail if tail else 0)
            nC = (nbytes + 15) // 16
            heads.add((nC + 1) % 64)
            pt = seedgen.data_np(59, nbytes, nbytes)
            want_ct, want_tag = O.gcm_encrypt(rk, nr, iv, aad, pt)
            ct, tag = gpu_encrypt(A, ws, rk, nr, iv, aad, pt)
            what = "%d bytes" % nbytes
            assert_same(ct, want_ct, what + " ciphertext")
            assert_same(tag, want_tag, what + " tag")
            back, ok = gpu_decrypt(A, ws, rk, nr, iv, aad, ct, tag)
            assert ok == 1, what
            assert_same(back, pt, what + " decrypt")
    assert heads == set(range(64))


@pytest.mark.parametrize("ivlen", [1, 8, 13, 16, 17, 60, 256])
def test_gcm_iv_lengths(A, O, ws, ivlen):
    rk, nr = A.aes_expand_key(seedgen.key(52, ivlen, 128))
    iv = seedgen.bytes_np(seedgen.stream_seed(52, seedgen.TAG_NONCE, ivlen), ivlen)
    pt = seedgen.data_np(52, ivlen, 5000)
    aad = seedgen.data_np(53, ivlen, 40)
    want_ct, want_tag = O.gcm_encrypt(rk, nr, iv, aad, pt)
    ct, tag = gpu_encrypt(A, ws, rk, nr, iv, aad, pt)
    assert_same(ct, want_ct, "IV %d B ciphertext" % ivlen)
    assert_same(tag, want_tag, "IV %d B tag" % ivlen)


def test_gcm_rejects_changes(A, O, ws):
    rk, nr = A.aes_expand_key(seedgen.key(54, 0, 256))
    iv = seedgen.nonce(54, 0)[:12]
    pt = seedgen.data_np(54, 0, 100000)
    aad = seedgen.data_np(54, 1, 64)
    ct, tag = gpu_encrypt(A, ws, rk, nr, iv, aad, pt)
    assert gpu_decrypt(A, ws, rk, nr, iv, aad, ct, tag[:12])[1] == 1        # truncated tag
    bad = ct.copy()
    bad[54321] ^= 4
    assert gpu_decrypt(A, ws, rk, nr, iv, aad, bad, tag)[1] == 0
    badtag = tag.copy()
    badtag[15] ^= 1
    assert gpu_decrypt(A, ws, rk, nr, iv, aad, ct, badtag)[1] == 0
    bada = aad.copy()
    bada[63] ^= 0x80
    assert gpu_decrypt(A, ws, rk, nr, iv, bada, ct, tag)[1] == 0
    # the oracle agrees on every verdict
    for c, t, a_ in ((ct, tag, aad), (bad, tag, aad), (ct, badtag, aad), (ct, tag, bada)):
        assert O.gcm_decrypt(rk, nr, iv, a_, c, t)[1] == (gpu_decrypt(A, ws, rk, nr, iv, a_, c, t)[1] == 1)


def test_gcm_in_place(A, O, ws):
    rk, nr = A.aes_expand_key(seedgen.key(55, 0, 128))
    iv = seedgen.nonce(55, 0)[:12]
    pt = seedgen.data_np(55, 0, 300001)
    aad = seedgen.data_np(55, 1, 16)
    want_ct, want_tag = O.gcm_encrypt(rk, nr, iv, aad, pt)
    x, ad = dev(pt), dev(aad)
    tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
    A.aes_gcm_encrypt(x, x, pt.size, ad, aad.size, rk, nr, iv, tag, ws)
    torch.cuda.synchronize()
    assert_same(x[:pt.size].cpu().numpy(), want_ct, "in place ciphertext")
    assert_same(tag.cpu().numpy(), want_tag, "in place tag")
    ok = torch.zeros(1, dtype=torch.int32, device="cuda")
    A.aes_gcm_decrypt(x, x, pt.size, ad, aad.size, rk, nr, iv, tag, 16, ok, ws)
    torch.cuda.synchronize()
    assert ok.item() == 1
    assert_same(x[:pt.size].cpu().numpy(), pt, "in place decrypt")


def test_gcm_16mib_whole(A, O, ws):
    # 2^20 blocks: the bulk kernel runs all 256 workgroups
    rk, nr = A.aes_expand_key(seedgen.key(56, 0, 128))
    iv = seedgen.nonce(56, 0)[:12]
    pt = seedgen.data_np(56, 0, (1 << 24) + 9)
    aad = seedgen.data_np(56, 1, 77)
    want_ct, want_tag = O.gcm_encrypt(rk, nr, iv, aad, pt)
    ct, tag = gpu_encrypt(A, ws, rk, nr, iv, aad, pt)
    assert_same(ct, want_ct, "16 MiB ciphertext")
    assert_same(tag, want_tag, "16 MiB tag")


@pytest.mark.parametrize("nbytes,aad_bytes", [(0, (1 << 24) + 5), ((1 << 20) + 3, (1 << 22) + 16)])
def test_gcm_long_additional_data(A, O, ws, nbytes, aad_bytes):
    # whole chunks of additional data take their own path (hash only): GMAC
    # over 16 MiB, and a message whose additional data outweighs it
    rk, nr = A.aes_expand_key(seedgen.key(58, 0, 256))
    iv = seedgen.nonce(58, 0)[:12]
    pt = seedgen.data_np(58, 1, nbytes)
    aad = seedgen.data_np(58, 2, aad_bytes)
    want_ct, want_tag = O.gcm_encrypt(rk, nr, iv, aad, pt)
    ct, tag = gpu_encrypt(A, ws, rk, nr, iv, aad, pt)
    assert_same(ct, want_ct, "long AAD ciphertext")
    assert_same(tag, want_tag, "long AAD tag")
    assert gpu_decrypt(A, ws, rk, nr, iv, aad, ct, tag)[1] == 1


def h_power(O, h, e):
    """H^e by square and multiply with the oracle's product."""
    one = np.zeros(16, np.uint8)
    one[0] = 0x80
    r, b = one, h.copy()
    while e:
        if e & 1:
            r = O.gcm_mul(r, b)
        b = O.gcm_mul(b, b)
        e >>= 1
    return r


def test_gcm_1gib_sampled(A, O, ws):
    n = 1 << 30
    rk, nr = A.aes_expand_key(seedgen.key(2, 0, 128))
    iv = seedgen.nonce(2, 3)[:12]
    x = seedgen.data_torch(2, 0, n, "cuda")
    y = torch.empty_like(x)
    aad = seedgen.data_np(57, 0, 48)
    ad = dev(aad)
    tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
    A.aes_gcm_encrypt(x, y, n, ad, aad.size, rk, nr, iv, tag, ws)
    torch.cuda.synchronize()
    t0 = tag.cpu().numpy()
    nblk = n // 16
    # ciphertext: CTR from J0 + 1, J0 = IV || 0^31 || 1
    j0 = np.concatenate([iv, np.array([0, 0, 0, 1], np.uint8)])
    rng = np.random.default_rng(9)
    idx = np.unique(np.concatenate([rng.integers(0, nblk, 256), [0, 1, nblk - 2, nblk - 1]]))
    got = y.view(-1, 16)[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    for r, j in enumerate(idx):
        p = seedgen.data_np(2, 0, 16, offset=16 * int(j))
        assert np.array_equal(got[r], O.ctr(rk, nr, j0, p, first_block=1 + int(j))), j
    # tag: flip one plaintext bit in block j; the tag moves by d * H^(nblk - j + 1)
    h = O.encrypt_block(rk, nr, np.zeros(16, np.uint8))
    for j in (0, 1, 4095, 4096, 1 << 20, nblk // 3, nblk - 257, nblk - 1):
        d = np.zeros(16, np.uint8)
        d[j % 16] = 1 << (j % 8)
        x.view(-1, 16)[j] ^= torch.from_numpy(d).to("cuda")
        A.aes_gcm_encrypt(x, y, n, ad, aad.size, rk, nr, iv, tag, ws)
        torch.cuda.synchronize()
        x.view(-1, 16)[j] ^= torch.from_numpy(d).to("cuda")
        moved = tag.cpu().numpy() ^ t0
        assert np.array_equal(moved, O.gcm_mul(d, h_power(O, h, nblk - j + 1))), "block %d" % j
    # additional data block k sits nblk + 1 + (blocks of A after k) positions from the end
    for k in (0, 2):
        d = np.zeros(16, np.uint8)
        d[3] = 0x10
        a2 = aad.copy()
        a2[16 * k:16 * k + 16] ^= d
        A.aes_gcm_encrypt(x, y, n, dev(a2), aad.size, rk, nr, iv, tag, ws)
        torch.cuda.synchronize()
        moved = tag.cpu().numpy() ^ t0
        assert np.array_equal(moved, O.gcm_mul(d, h_power(O, h, nblk + 1 + (3 - k)))), "AAD block %d" % k
    # and the whole buffer round trip with the tag check
    ok = torch.zeros(1, dtype=torch.int32, device="cuda")
    z = torch.empty_like(x)
    A.aes_gcm_encrypt(x, y, n, ad, aad.size, rk, nr, iv, tag, ws)
    A.aes_gcm_decrypt(y, z, n, ad, aad.size, rk, nr, iv, tag, 16, ok, ws)
    torch.cuda.synchronize()
    assert ok.item() == 1
    assert torch.equal(z, x)
    del x, y, z
    torch.cuda.empty_cache()
