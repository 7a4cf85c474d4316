"""Parity of the HIP path with the oracle, bit for bit, through the C ABI.

AES output is fully determined by (key, mode, counter block, input), so the
tolerance everywhere is zero: every compared byte must be equal.  Small and
ragged sizes are compared in full.  The 1 GiB buffer of the throughput
workload is compared in full too (ECB encryption, ECB decryption of random
input, CTR), streamed through the oracle 64 MiB at a time; the 4 GiB buffers
are compared on sampled blocks that the oracle computes one by one, and in
full against the independent bitsliced kernel.
"""
import os

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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_op(A, op, x_np, rk, nr, ctr0=None, inplace=False, stream=None):
    """Run one operation ('enc' / 'dec' in ECB, or 'ctr') on the GPU; returns numpy."""
    x = to_dev(x_np)
    out = x if inplace else torch.empty_like(x)
    n = x_np.size
    if op == "enc":
        A.aes_encrypt(x, out, n, rk, nr, "ecb", stream=stream)
    elif op == "dec":
        A.aes_decrypt(x, out, n, rk, nr, "ecb", stream=stream)
    elif op == "ctr":
        A.aes_encrypt(x, out, n, rk, nr, "ctr", ctr0=ctr0, stream=stream)
    elif op == "ctr_dec":
        A.aes_decrypt(x, out, n, rk, nr, "ctr", ctr0=ctr0, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_op(O, op, x_np, rk, nr, ctr0=None):
    if op == "enc":
        return O.ecb_encrypt(rk, nr, x_np)
    if op == "dec":
        return O.ecb_decrypt(rk, nr, x_np)
    return O.ctr(rk, nr, ctr0, x_np)


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError("%s: %d bytes differ, first at %d (block %d)"
                             % (what, bad.size, bad[0], bad[0] // 16))


# --- C1: AES-128 ECB encrypt then decrypt, 1 MiB, whole buffer -------------
def test_c1_ecb_1mib(A, O):
    k = seedgen.key(1, 0, 128)
    rk, nr = A.aes_expand_key(k)
    x = seedgen.data_np(1, 0, 1 << 20)
    ct = gpu_op(A, "enc", x, rk, nr)
    assert_same(ct, O.ecb_encrypt(rk, nr, x), "C1 encrypt")
    pt = gpu_op(A, "dec", ct, rk, nr)
    assert_same(pt, x, "C1 decrypt(encrypt(x))")


SIZES = [16, 4096, 65535 * 16, (1 << 20) + 48]
# CTR takes any length; ECB lengths that are not whole blocks are an argument
# error, checked on the host (test_abi_host)
CTR_ONLY_SIZES = [1, 15, 17, 31, 1000003]
SIZE_CASES = [(n, op) for n in SIZES for op in ("enc", "dec", "ctr", "ctr_dec")] + \
             [(n, op) for n in CTR_ONLY_SIZES for op in ("ctr", "ctr_dec")]


@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("nbytes,op", SIZE_CASES)
def test_sizes(A, O, bits, op, nbytes):
    seed = 1000 * bits + nbytes
    k = seedgen.key(3, seed, bits)
    rk, nr = A.aes_expand_key(k)
    x = seedgen.data_np(3, seed, nbytes)
    ctr0 = seedgen.nonce(3, seed)
    got = gpu_op(A, op, x, rk, nr, ctr0=ctr0)
    assert_same(got, oracle_op(O, op, x, rk, nr, ctr0), "%s AES-%d %d bytes" % (op, bits, nbytes))


def test_empty_buffer(A):
    rk, nr = A.aes_expand_key(bytes(16))
    x = torch.empty(0, dtype=torch.uint8, device="cuda")
    A.aes_encrypt(x, x, 0, rk, nr, "ecb")
    A.aes_decrypt(x, x, 0, rk, nr, "ctr", ctr0=bytes(16))
    torch.cuda.synchronize()


@pytest.mark.parametrize("op", ["enc", "dec", "ctr"])
def test_in_place_equals_out_of_place(A, O, op):
    k = seedgen.key(4, 0, 256)
    rk, nr = A.aes_expand_key(k)
    x = seedgen.data_np(4, 0, 300000 * 16 + (0 if op != "ctr" else 7))
    ctr0 = seedgen.nonce(4, 0)
    a = gpu_op(A, op, x, rk, nr, ctr0=ctr0)
    b = gpu_op(A, op, x, rk, nr, ctr0=ctr0, inplace=True)
    assert_same(b, a, "in place vs out of place")
    assert_same(a, oracle_op(O, op, x, rk, nr, ctr0), "oracle")


def test_ctr_counter_wraps_without_carry(A, O):
    k = seedgen.key(5, 0, 128)
    rk, nr = A.aes_expand_key(k)
    ctr0 = seedgen.nonce(5, 0)
    ctr0[12:16] = [0xFF, 0xFF, 0xFF, 0xF0]
    x = seedgen.data_np(5, 0, 16 * 5000 + 3)
    got = gpu_op(A, "ctr", x, rk, nr, ctr0=ctr0)
    assert_same(got, O.ctr(rk, nr, ctr0, x), "CTR across the 2^32 wrap")


# every table layout (four tables x 32 copies, two x 64, one x 64 with
# rotations, four unreplicated), blocks per thread, workgroup size, and the
# default grid (as many workgroups as fit per compute unit), one workgroup,
# or seven
LAUNCHES = [dict(layout=l, blocks_per_thread=b, wg_size=w, grid=g)
            for l in (0, 1, 3, 4) for b in (1, 2, 4) for w in (256, 1024) for g in (0, 1, 7)]


@pytest.fixture(scope="module")
def ragged_case(A, O):
    k = seedgen.key(6, 0, 128)
    rk, nr = A.aes_expand_key(k)
    x = seedgen.data_np(6, 0, 3 * 65536 * 16 + 48 + 5)
    ctr0 = seedgen.nonce(6, 0)
    n16 = x.size - 5
    want = {"enc": O.ecb_encrypt(rk, nr, x[:n16]), "dec": O.ecb_decrypt(rk, nr, x[:n16]),
            "ctr": O.ctr(rk, nr, ctr0, x)}
    return rk, nr, x, n16, ctr0, want


@pytest.mark.parametrize("cfg", LAUNCHES, ids=lambda c: "L%d-B%d-W%d-G%d" % tuple(c.values()))
def test_launch_configurations_agree(A, ragged_case, cfg):
    rk, nr, x, n16, ctr0, want = ragged_case
    A.aes_set_launch(cfg)
    try:
        assert_same(gpu_op(A, "enc", x[:n16], rk, nr), want["enc"], "enc %s" % cfg)
        assert_same(gpu_op(A, "dec", x[:n16], rk, nr), want["dec"], "dec %s" % cfg)
        assert_same(gpu_op(A, "ctr", x, rk, nr, ctr0=ctr0), want["ctr"], "ctr %s" % cfg)
    finally:
        A.aes_set_launch(None)


@pytest.mark.parametrize("start", [1, 0x80, 0xFF, 0xFFFFFF81], ids=lambda v: "c%08x" % v)
def test_ctr_unaligned_counter_starts(A, O, start):
    """CTR whose 32-bit counter starts off a multiple of 256: every step of
    256 blocks then crosses one, and the blocks on either side share
    different round-1 columns (the last start also crosses the 2^32 wrap).
    Every table layout at four blocks per thread, default grid and seven
    workgroups, against the oracle on a ragged 1 MiB buffer."""
    k = seedgen.key(9, start & 0xFF, 128)
    rk, nr = A.aes_expand_key(k)
    x = seedgen.data_np(9, 1, (1 << 20) + 21)
    ctr0 = seedgen.nonce(9, 2)
    ctr0[12:16] = list(int(start).to_bytes(4, "big"))
    want = O.ctr(rk, nr, ctr0, x)
    for layout in (0, 1, 3, 4):
        for grid in (0, 7):
            cfg = dict(layout=layout, blocks_per_thread=4, wg_size=1024, grid=grid)
            A.aes_set_launch(cfg)
            try:
                assert_same(gpu_op(A, "ctr", x, rk, nr, ctr0=ctr0), want, "ctr from %#x %s" % (start, cfg))
            finally:
                A.aes_set_launch(None)


def test_side_stream(A, O):
    k = seedgen.key(7, 0, 256)
    rk, nr = A.aes_expand_key(k)
    x = seedgen.data_np(7, 0, 1 << 18)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = gpu_op(A, "enc", x, rk, nr, stream=s)
    assert_same(got, O.ecb_encrypt(rk, nr, x), "side stream")


def test_device_errors(A):
    rk, nr = A.aes_expand_key(bytes(16))
    x = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(A.AESError) as e:
        A.aes_encrypt(x[1:], x[1:], 1024, rk, nr, "ecb")
    assert e.value.code == A.AES_E_ALIGN
    with pytest.raises(A.AESError) as e:
        A.aes_encrypt(x[:1024], x[16:], 1024, rk, nr, "ecb")
    assert e.value.code == A.AES_E_OVERLAP


def test_copy_helper(A):
    x = seedgen.data_torch(8, 0, (1 << 20) + 16 * 3, "cuda")
    y = torch.empty_like(x)
    A.aes_copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def lds_gather_folds(blocks, rounds, layout=0):
    """What each workgroup of the LDS calibration kernel must report: word i
    of the LDS holds i * 0x9E3779B1; lane l of workgroup b starts column word
    c at (l + 64 c + 1) * 0x9E3779B1 ^ b, adds 0x3B5D7F91 + c per round and
    reads, in table K, entry byte K of that word, copy l & 31 (layout 0), or
    that entry of the one table, copy l (layout 3); the wave's fold is the
    XOR of every word read and of the lane numbers."""
    m = np.uint64(0xFFFFFFFF)
    phi = np.uint64(0x9E3779B1)
    lane = np.arange(64, dtype=np.uint64)[None, :]
    b = np.arange(blocks, dtype=np.uint64)[:, None]
    if layout == 3:
        lc = [lane << np.uint64(2) for t in range(4)]
    else:
        lc = [((lane & np.uint64(31)) << np.uint64(2)) | np.uint64((t & 1) << 7) | np.uint64((t >> 1) << 16)
              for t in range(4)]
    w = [(((lane + np.uint64(64 * c + 1)) * phi) & m) ^ b for c in range(4)]
    acc = np.zeros((blocks, 64), np.uint64)
    for _ in range(rounds):
        for c in range(4):
            w[c] = (w[c] + np.uint64(0x3B5D7F91 + c)) & m
            for k in range(4):
                addr = lc[k] | (((w[c] >> np.uint64(8 * k)) & np.uint64(0xFF)) << np.uint64(8))
                acc ^= ((addr >> np.uint64(2)) * phi) & m
    acc ^= lane
    return np.bitwise_xor.reduce(acc, axis=1)


def test_lds_gather_helper(A):
    """The LDS calibration kernel: one record per wave, both clocks advance,
    and every wave's fold of the words it read is the one computed here."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    waves = cus * 16
    rounds = 64
    rec = torch.full((waves * 3,), -1, dtype=torch.int64, device="cuda")
    w, khz = A.aes_lds_gather(rec, rounds)
    torch.cuda.synchronize()
    assert w == waves and khz > 0
    r = rec.view(-1, 3).cpu().numpy()
    assert (r[:, 0] > 0).all() and (r[:, 1] > 0).all()
    fold = r[:, 2].astype(np.uint64)
    expect = np.repeat(lds_gather_folds(cus, rounds), 16)     # 16 waves per workgroup read alike
    assert np.array_equal(fold, expect)                         # fold in the low word, pad (0) above
    with pytest.raises(A.AESError) as e:
        A.aes_lds_gather(rec[:3], rounds)
    assert e.value.code == A.AES_E_LENGTH
    with pytest.raises(A.AESError) as e:
        A.aes_lds_gather(rec, 0)
    assert e.value.code == A.AES_E_ARG
    # the one-table layout: two workgroups per compute unit, copy = lane
    rec2 = torch.full((2 * waves * 3,), -1, dtype=torch.int64, device="cuda")
    w2, _ = A.aes_lds_gather(rec2, rounds, layout=3)
    torch.cuda.synchronize()
    assert w2 == 2 * waves
    fold2 = rec2.view(-1, 3).cpu().numpy()[:, 2].astype(np.uint64)
    assert np.array_equal(fold2, np.repeat(lds_gather_folds(2 * cus, rounds, layout=3), 16))
    with pytest.raises(A.AESError) as e:
        A.aes_lds_gather(rec2, rounds, layout=1)
    assert e.value.code == A.AES_E_ARG


def test_device_generator_matches_host(A):
    for n in (1, 1000, (1 << 22) + 5):
        d = seedgen.data_torch(9, 1, n, "cuda").cpu().numpy()
        assert np.array_equal(d, seedgen.data_np(9, 1, n))


# --- full sizes, sampled -------------------------------------------------
def sample_blocks(nblocks, count, seed):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, nblocks, size=count)
    return np.unique(np.concatenate([idx, [0, 1, nblocks - 2, nblocks - 1]]))


def check_sampled(O, out_dev, master, index, rk, nr, op, ctr0, idx, what):
    got = out_dev.view(-1, 16)[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    for r, j in enumerate(idx):
        x = seedgen.data_np(master, index, 16, offset=16 * int(j))
        if op == "enc":
            want = O.encrypt_block(rk, nr, x)
        elif op == "dec":
            want = O.decrypt_block(rk, nr, x)
        else:
            want = O.ctr(rk, nr, ctr0, x, first_block=int(j))
        if not np.array_equal(got[r], want):
            raise AssertionError("%s: block %d differs" % (what, j))


@pytest.mark.parametrize("bits,nbytes,ops", [
    (128, 1 << 30, ("enc", "ctr")),          # the throughput workload: 1 GiB, AES-128
    (256, 1 << 24, ("enc", "ctr")),
    (256, 1 << 28, ("enc", "ctr")),
    (256, 1 << 32, ("enc", "ctr")),
], ids=["aes128-1GiB", "aes256-16MiB", "aes256-256MiB", "aes256-4GiB"])
def test_full_size_sampled(A, O, bits, nbytes, ops):
    master, index = 2 if bits == 128 else 3, 0
    k = seedgen.key(master, index, bits)
    rk, nr = A.aes_expand_key(k)
    ctr0 = seedgen.nonce(master, index)
    x = seedgen.data_torch(master, index, nbytes, "cuda")
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    idx = sample_blocks(nbytes // 16, 2048, nbytes)
    for op in ops:
        mode = "ecb" if op == "enc" else "ctr"
        A.aes_encrypt(x, y, nbytes, rk, nr, mode, ctr0=ctr0)
        torch.cuda.synchronize()
        check_sampled(O, y, master, index, rk, nr, op, ctr0, idx, "%s %d bytes" % (op, nbytes))
        if op == "enc":
            # the decryption kernel on its own, applied to the random input
            A.aes_decrypt(x, z, nbytes, rk, nr, mode)
            torch.cuda.synchronize()
            check_sampled(O, z, master, index, rk, nr, "dec", ctr0, idx, "dec %d bytes" % nbytes)
        A.aes_decrypt(y, z, nbytes, rk, nr, mode, ctr0=ctr0)
        torch.cuda.synchronize()
        assert torch.equal(z, x), "%s: decrypt(encrypt(x)) != x" % op
    del x, y, z
    torch.cuda.empty_cache()


def test_aes256_16mib_whole_buffer(A, O):
    k = seedgen.key(3, 0, 256)
    rk, nr = A.aes_expand_key(k)
    ctr0 = seedgen.nonce(3, 0)
    x = seedgen.data_np(3, 0, 1 << 24)
    want, _ = O.par_run(0, rk, nr, x, 16)
    assert_same(gpu_op(A, "enc", x, rk, nr), want, "AES-256 ECB 16 MiB")
    want, _ = O.par_run(2, rk, nr, x, 16, ctr0=ctr0)
    assert_same(gpu_op(A, "ctr", x, rk, nr, ctr0=ctr0), want, "AES-256 CTR 16 MiB")


# --- the bitsliced comparison kernel (launch layout 2) ----------------------
@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("grid", [0, 1, 7])
def test_bitsliced_matches_oracle(A, O, bits, grid):
    k = seedgen.key(11, bits, bits)
    rk, nr = A.aes_expand_key(k)
    x = seedgen.data_np(11, bits, 5 * 2048 * 16 + 777 * 16 + 9)   # several waves' worth and a ragged tail
    ctr0 = seedgen.nonce(11, bits)
    ctr0[12:16] = [0x00, 0x00, 0xFF, 0x80]                        # counter crosses byte boundaries
    n16 = x.size - 9
    A.aes_set_launch(layout=2, grid=grid)
    try:
        assert_same(gpu_op(A, "enc", x[:n16], rk, nr), O.ecb_encrypt(rk, nr, x[:n16]), "bitsliced ECB")
        assert_same(gpu_op(A, "ctr", x, rk, nr, ctr0=ctr0), O.ctr(rk, nr, ctr0, x), "bitsliced CTR")
        assert_same(gpu_op(A, "ctr_dec", x[:100], rk, nr, ctr0=ctr0), O.ctr(rk, nr, ctr0, x[:100]),
                    "bitsliced CTR decrypt")
        with pytest.raises(A.AESError) as e:
            gpu_op(A, "dec", x[:n16], rk, nr)
        assert e.value.code == A.AES_E_ARG
    finally:
        A.aes_set_launch(None)


@pytest.mark.parametrize("bits,n", [(128, 1 << 30), (256, 1 << 32)], ids=["aes128-1GiB", "aes256-4GiB"])
def test_bitsliced_equals_table_kernel_whole_buffer(A, O, bits, n):
    """Two independent kernels (round tables in LDS; a Boolean S-box circuit
    on bit-planes) agree on every byte of the 1 GiB and 4 GiB workloads."""
    master = 2 if bits == 128 else 3
    k = seedgen.key(master, 0, bits)
    rk, nr = A.aes_expand_key(k)
    ctr0 = seedgen.nonce(master, 0)
    x = seedgen.data_torch(master, 0, n, "cuda")
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    for mode in ("ecb", "ctr"):
        A.aes_encrypt(x, y, n, rk, nr, mode, ctr0=ctr0)
        A.aes_set_launch(layout=2)
        try:
            A.aes_encrypt(x, z, n, rk, nr, mode, ctr0=ctr0)
        finally:
            A.aes_set_launch(None)
        torch.cuda.synchronize()
        assert torch.equal(y, z), mode
    idx = sample_blocks(n // 16, 256, 7)
    check_sampled(O, z, master, 0, rk, nr, "ctr", ctr0, idx, "bitsliced CTR %d bytes" % n)
    del x, y, z
    torch.cuda.empty_cache()


def ctr_block_offset(ctr0, j):
    """The counter block of block j: the nonce bytes, then the 32-bit
    big-endian counter advanced by j modulo 2^32 (no carry into the nonce)."""
    c = np.array(ctr0, dtype=np.uint8).copy()
    v = (int.from_bytes(bytes(c[12:16]), "big") + j) & 0xFFFFFFFF
    c[12:16] = np.frombuffer(v.to_bytes(4, "big"), np.uint8)
    return c


@pytest.mark.parametrize("op", ["enc", "dec", "ctr"])
def test_headline_buffer_whole_against_oracle(A, O, op):
    """Every byte of the 1 GiB AES-128 throughput workload, computed in the
    launch configuration the benchmark times, against the oracle: the input
    is regenerated on the host 64 MiB at a time and the oracle runs the
    paper's method on it (one contiguous chunk per host thread)."""
    master, index, n, chunk = 2, 0, 1 << 30, 1 << 26
    k = seedgen.key(master, index, 128)
    rk, nr = A.aes_expand_key(k)
    ctr0 = seedgen.nonce(master, index)
    x = seedgen.data_torch(master, index, n, "cuda")
    y = torch.empty_like(x)
    if op == "dec":
        A.aes_decrypt(x, y, n, rk, nr, "ecb")
    else:
        A.aes_encrypt(x, y, n, rk, nr, "ecb" if op == "enc" else "ctr", ctr0=ctr0)
    torch.cuda.synchronize()
    del x
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    opcode = {"enc": ref.OP_ECB_ENC, "dec": ref.OP_ECB_DEC, "ctr": ref.OP_CTR}[op]
    for off in range(0, n, chunk):
        xc = seedgen.data_np(master, index, chunk, offset=off)
        c0 = ctr_block_offset(ctr0, off // 16) if op == "ctr" else None
        want, _ = O.par_run(opcode, rk, nr, xc, threads, ctr0=c0)
        assert_same(y[off:off + chunk].cpu().numpy(), want, "%s 1 GiB, chunk at %d" % (op, off))
    del y
    torch.cuda.empty_cache()


# --- CBC ----------------------------------------------------------------
@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("nbytes", [16, 4096, 65535 * 16, (1 << 20) + 48])
def test_cbc_decrypt_matches_oracle(A, O, bits, nbytes):
    seed = 7000 + bits + nbytes
    rk, nr = A.aes_expand_key(seedgen.key(12, seed, bits))
    iv = seedgen.bytes_np(seedgen.stream_seed(12, seedgen.TAG_NONCE, seed), 16)
    x = seedgen.data_np(12, seed, nbytes)
    assert_same(gpu_op_cbc(A, False, x, rk, nr, iv), O.cbc_decrypt(rk, nr, iv, x),
                "CBC decrypt AES-%d %d bytes" % (bits, nbytes))


@pytest.mark.parametrize("bits", [128, 256])
# 1, 3, 5, 7 blocks: partial groups of the four blocks read ahead, first and later
@pytest.mark.parametrize("nbytes", [16, 48, 80, 112, 4096, 1 << 18])
def test_cbc_encrypt_matches_oracle(A, O, bits, nbytes):
    seed = 8000 + bits + nbytes
    rk, nr = A.aes_expand_key(seedgen.key(13, seed, bits))
    iv = seedgen.bytes_np(seedgen.stream_seed(13, seedgen.TAG_NONCE, seed), 16)
    x = seedgen.data_np(13, seed, nbytes)
    want = O.cbc_encrypt(rk, nr, iv, x)
    assert_same(gpu_op_cbc(A, True, x, rk, nr, iv), want, "CBC encrypt")
    assert_same(gpu_op_cbc(A, True, x, rk, nr, iv, inplace=True), want, "CBC encrypt in place")


def gpu_op_cbc(A, encrypt, x_np, rk, nr, iv, inplace=False):
    x = to_dev(x_np)
    out = x if inplace else torch.empty_like(x)
    (A.aes_encrypt if encrypt else A.aes_decrypt)(x, out, x_np.size, rk, nr, "cbc", ctr0=iv)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("cfg", [dict(layout=l, blocks_per_thread=b, wg_size=w, grid=g)
                                 for l in (0, 1) for b in (1, 4) for w in (256, 1024) for g in (0, 3)],
                         ids=lambda c: "L%d-B%d-W%d-G%d" % tuple(c.values()))
def test_cbc_decrypt_launch_configurations(A, O, cfg):
    rk, nr = A.aes_expand_key(seedgen.key(14, 0, 128))
    iv = seedgen.nonce(14, 0)
    x = seedgen.data_np(14, 0, 3 * 65536 * 16 + 48)
    want = O.cbc_decrypt(rk, nr, iv, x)
    A.aes_set_launch(cfg)
    try:
        assert_same(gpu_op_cbc(A, False, x, rk, nr, iv), want, "CBC decrypt %s" % cfg)
    finally:
        A.aes_set_launch(None)


def test_cbc_decrypt_1gib_sampled(A, O):
    rk, nr = A.aes_expand_key(seedgen.key(2, 0, 128))
    iv = seedgen.nonce(2, 1)
    n = 1 << 30
    x = seedgen.data_torch(2, 0, n, "cuda")
    y = torch.empty_like(x)
    A.aes_decrypt(x, y, n, rk, nr, "cbc", ctr0=iv)
    torch.cuda.synchronize()
    idx = sample_blocks(n // 16, 1024, 11)
    got = y.view(-1, 16)[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    for r, j in enumerate(idx):
        c = seedgen.data_np(2, 0, 16, offset=16 * int(j))
        prev = iv if j == 0 else seedgen.data_np(2, 0, 16, offset=16 * (int(j) - 1))
        assert np.array_equal(got[r], O.cbc_decrypt(rk, nr, prev, c)), j
    # and the round trip through the serial encryption on a slice
    z = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    A.aes_encrypt(y[:1 << 16], z, 1 << 16, rk, nr, "cbc", ctr0=iv)
    torch.cuda.synchronize()
    assert torch.equal(z, x[:1 << 16])
