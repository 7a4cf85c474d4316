"""The batched path (on-device key expansion, the plan that splits the work
into one share per wave, persistent kernels, graph replay) against the oracle
and against the single-buffer path, bit for bit, through the C ABI."""
import numpy as np
import pytest

import seedgen
from oracle import ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SENTINEL = 0xA5


@pytest.fixture(scope="module")
def A():
    from paper_1403_7295_amd import aesgpu
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return aesgpu


@pytest.fixture(scope="module")
def O():
    return ref.default()


def mixed_messages(A, n, seed, max_len=1 << 16, min_len=0, mode=None, decrypt=None, modes=4):
    """n messages of every kind: ECB encrypt/decrypt, CTR, CBC and XTS
    encrypt/decrypt (the first `modes` modes), 128/192/256-bit keys, lengths
    log-uniform in [1, max_len] (all but CTR rounded up to whole blocks), a
    few empty ones (unless min_len > 0), counters that wrap, XTS data units of
    16 B .. 4 KiB with the tweak key in another message's key slot."""
    rng = np.random.default_rng(seed)
    lens = np.maximum(seedgen.log_uniform_lengths(rng, n, 1, max_len), min_len)
    mode = rng.integers(0, modes, n) if mode is None else np.full(n, mode)
    decrypt = rng.integers(0, 2, n) if decrypt is None else np.full(n, decrypt)
    keybits = rng.choice([128, 192, 256], n)
    lens = np.where(mode != 1, (lens + 15) // 16 * 16, lens)
    if min_len == 0:
        lens[rng.choice(n, 3, replace=False)] = 0
    keys = np.zeros((n, 32), np.uint8)
    ctr0 = np.zeros((n, 16), np.uint8)
    units = rng.choice([16, 32, 512, 4096], n)
    for m in range(n):
        keys[m, :keybits[m] // 8] = seedgen.key(seed, m, int(keybits[m]))
        ctr0[m] = seedgen.nonce(seed, m)
        if m % 7 == 0:
            ctr0[m, 12:16] = [0xFF, 0xFF, 0xFF, 0xF8]   # wraps inside the message
        if mode[m] == 3:
            first = int(rng.integers(0, 1 << 62)) if m % 3 else (1 << 64) - 5   # and one that wraps
            ctr0[m] = A.xts_ctr0(first, (m + 1) % n, int(units[m]))
    descs = A.make_descs(lens, keybits=keybits, mode=mode, decrypt=decrypt, ctr0=ctr0)
    return descs, keys


def buffers(descs, seed):
    end = int((descs["in_off"] + descs["nbytes"]).max()) if len(descs) else 0
    total = (end + 15) // 16 * 16 + 16
    x = seedgen.data_np(seed, 99, total)
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.full_like(xd, SENTINEL)
    return x, xd, yd


def xts_fields(d):
    c = bytes(d["ctr0"])
    return (int.from_bytes(c[0:8], "little"), int.from_bytes(c[8:12], "little"),
            int.from_bytes(c[12:16], "little"))


def oracle_message(O, d, keys, x):
    bits = 128 + 64 * int(d["keybits_code"])
    rk, nr = O.expand_key(keys[int(d["key_idx"])][:bits // 8])
    if d["mode"] == 3:
        first, key2, unit = xts_fields(d)
        rk2, _ = O.expand_key(keys[key2][:bits // 8])
        return O.xts(bool(d["decrypt"]), rk, rk2, nr, unit, first, x)
    if d["mode"] == 0:
        return O.ecb_decrypt(rk, nr, x) if d["decrypt"] else O.ecb_encrypt(rk, nr, x)
    if d["mode"] == 2:
        return O.cbc_decrypt(rk, nr, d["ctr0"], x) if d["decrypt"] else O.cbc_encrypt(rk, nr, d["ctr0"], x)
    return O.ctr(rk, nr, d["ctr0"], x)


def check_against_oracle(O, descs, keys, x, y):
    for m, d in enumerate(descs):
        n = int(d["nbytes"])
        i, o = int(d["in_off"]), int(d["out_off"])
        want = oracle_message(O, d, keys, x[i:i + n])
        if not np.array_equal(y[o:o + n], want):
            raise AssertionError("message %d (%s) differs" % (m, d))


def test_batch_matches_oracle(A, O):
    descs, keys = mixed_messages(A, 300, 41)
    x, xd, yd = buffers(descs, 41)
    b = A.Batch(descs, keys, xd, yd)
    b.run()
    planned, rejected = b.query()
    assert rejected == 0 and planned > 0
    check_against_oracle(O, descs, keys, x, yd.cpu().numpy())


@pytest.mark.parametrize("tile_blocks", [1, 64, 777, 1024])
def test_split_granularity_and_order_do_not_matter(A, tile_blocks):
    descs, keys = mixed_messages(A, 120, 42, max_len=1 << 18)
    x, xd, y0 = buffers(descs, 42)
    A.Batch(descs, keys, xd, y0).run()
    y1 = torch.full_like(y0, SENTINEL)
    perm = np.random.default_rng(tile_blocks).permutation(len(descs))
    A.Batch(descs[perm], keys, xd, y1, tile_blocks=tile_blocks).run()
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)


@pytest.mark.parametrize("bpt", [2, 4])
def test_blocks_per_thread_matches_oracle(A, O, bpt):
    # both block-loop widths the autotuner chooses between, every mode
    descs, keys = mixed_messages(A, 150, 46, max_len=1 << 18)
    x, xd, yd = buffers(descs, 46)
    b = A.Batch(descs, keys, xd, yd, blocks_per_thread=bpt)
    assert b.c.blocks_per_thread == bpt
    b.run()
    assert b.query()[1] == 0
    check_against_oracle(O, descs, keys, x, yd.cpu().numpy())


def test_in_place(A, O):
    descs, keys = mixed_messages(A, 50, 43, modes=2)   # CBC decryption cannot run in place
    x, xd, _ = buffers(descs, 43)
    A.Batch(descs, keys, xd, xd).run()
    check_against_oracle(O, descs, keys, x, xd.cpu().numpy())


def test_graph_replay_with_rewritten_descriptors(A, O):
    descs, keys = mixed_messages(A, 80, 44)
    x, xd, yd = buffers(descs, 44)
    b = A.Batch(descs, keys, xd, yd, max_msgs=80)
    for rep in range(3):
        yd.fill_(SENTINEL)
        b.launch_graph()
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        check_against_oracle(O, descs, keys, x, yd.cpu().numpy())
    # fewer messages, new keys: the graph reads the count from the device
    descs2, keys2 = mixed_messages(A, 30, 45)
    descs2["in_off"] = descs["in_off"][:30]
    descs2["out_off"] = descs["out_off"][:30]
    descs2["nbytes"] = np.minimum(descs2["nbytes"], descs["nbytes"][:30])
    descs2["nbytes"] = np.where(descs2["mode"] != 1, descs2["nbytes"] // 16 * 16, descs2["nbytes"])
    b.set_descs(descs2, keys2)
    yd.fill_(SENTINEL)
    b.launch_graph()
    torch.cuda.synchronize()
    check_against_oracle(O, descs2, keys2, x, yd.cpu().numpy())
    b.close()


def test_invalid_descriptors_are_skipped(A, O):
    descs, keys = mixed_messages(A, 40, 46, min_len=32)
    bad = descs.copy()
    bad["keybits_code"][0] = 3                     # no such key size
    bad["mode"][1] = 0
    bad["nbytes"][1] = 17                          # ECB, not whole blocks
    bad["in_off"][2] += 8                          # misaligned
    bad["key_idx"][3] = len(keys)                  # no such key
    x, xd, yd = buffers(descs, 46)
    bad["nbytes"][4] = xd.numel() + 16             # outside the buffers
    for m, (unit, key2, nbytes) in zip((5, 6, 7), ((24, 0, 64), (512, len(keys), 64), (512, 0, 40))):
        bad["mode"][m] = 3                         # XTS: unit not a power of two, no such
        bad["ctr0"][m] = A.xts_ctr0(0, key2, unit)  # tweak key, not whole blocks
        bad["nbytes"][m] = nbytes
    b = A.Batch(bad, keys, xd, yd)
    b.run()
    planned, rejected = b.query()
    assert rejected == 8 and planned == len(bad) - 8
    y = yd.cpu().numpy()
    for m in range(8):
        o, n = int(descs["out_off"][m]), int(descs["nbytes"][m])
        assert (y[o:o + n] == SENTINEL).all(), "rejected message %d was written" % m
    check_against_oracle(O, descs[8:], keys, x, y)


@pytest.mark.parametrize("kind", ["ctr", "xts", "ecb_dec", "cbc_dec"])
def test_one_message_is_split_over_every_wave(A, O, kind):
    """A single message in a batch: the plan splits it over all the cipher
    kernel's waves (thousands of shares, each a few blocks), and the result
    is the oracle's."""
    n = 2 * 1024 * 1024 + (5 if kind == "ctr" else 0)
    mode = {"ctr": 1, "xts": 3, "ecb_dec": 0, "cbc_dec": 2}[kind]
    keys = np.zeros((2, 32), np.uint8)
    keys[0, :16] = seedgen.key(48, 0, 128)
    keys[1, :16] = seedgen.key(48, 1, 128)
    ctr0 = A.xts_ctr0(1000, 1, 512) if kind == "xts" else seedgen.nonce(48, 0)
    descs = A.make_descs([n], keybits=128, mode=mode, decrypt=kind in ("ecb_dec", "cbc_dec"), ctr0=ctr0)
    x, xd, yd = buffers(descs, 48)
    b = A.Batch(descs, keys, xd, yd)
    b.run()
    planned, rejected = b.query()
    assert (planned, rejected) == (1, 0)
    check_against_oracle(O, descs, keys, x, yd.cpu().numpy())


def test_many_tiny_messages(A, O):
    """More messages than waves, most of them one or two blocks, some empty:
    shares hold many messages each."""
    rng = np.random.default_rng(49)
    n = 6000
    lens = rng.integers(0, 3, n) * 16 + np.where(rng.random(n) < 0.3, rng.integers(1, 16, n), 0)
    mode = np.where(lens % 16 != 0, 1, rng.integers(0, 2, n))
    keybits = rng.choice([128, 256], n)
    keys = np.zeros((n, 32), np.uint8)
    for m in range(n):
        keys[m, :keybits[m] // 8] = seedgen.key(49, m, int(keybits[m]))
    descs = A.make_descs(lens, keybits=keybits, mode=mode, decrypt=rng.integers(0, 2, n),
                         ctr0=seedgen.nonce(49, 0))
    x, xd, yd = buffers(descs, 49)
    b = A.Batch(descs, keys, xd, yd)
    b.run()
    planned, rejected = b.query()
    assert (planned, rejected) == (n, 0)
    check_against_oracle(O, descs, keys, x, yd.cpu().numpy())


def test_empty_messages_only(A):
    descs = A.make_descs([0, 0, 0], mode=["ecb", "ctr", "cbc"], decrypt=[1, 0, 0])
    keys = np.zeros((3, 32), np.uint8)
    xd = torch.zeros(64, dtype=torch.uint8, device="cuda")
    yd = torch.full_like(xd, SENTINEL)
    b = A.Batch(descs, keys, xd, yd)
    b.run()
    assert b.query() == (3, 0)
    assert (yd.cpu().numpy() == SENTINEL).all()


def test_batch_equals_plain_on_ragged_workload(A, O):
    """The ragged multi-message workload at full size (10,000 messages,
    log-uniform 16 B .. 16 MiB, half AES-128, half AES-256, ECB encrypt):
    batched output equals per-message single-buffer launches byte for byte,
    and sampled blocks equal the oracle."""
    lens, keybits, keys, _ = seedgen.ragged_batch(4, 10000)
    descs = A.make_descs(lens, keybits=keybits, mode="ecb")
    total = int(lens.sum())
    x = seedgen.data_torch(4, 0, total, "cuda")
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    b = A.Batch(descs, keys, x, y)
    b.launch_graph()
    for m in range(len(descs)):
        o, n = int(descs["in_off"][m]), int(lens[m])
        rk, nr = A.aes_expand_key(keys[m][:keybits[m] // 8])
        A.aes_encrypt(x[o:o + n], z[o:o + n], n, rk, nr, "ecb")
    torch.cuda.synchronize()
    assert torch.equal(y, z)
    rng = np.random.default_rng(5)
    for m in rng.choice(len(descs), 300, replace=False):
        o, nblk = int(descs["in_off"][m]), int(lens[m]) // 16
        j = int(rng.integers(0, nblk))
        rk, nr = O.expand_key(keys[m][:keybits[m] // 8])
        want = O.encrypt_block(rk, nr, seedgen.data_np(4, 0, 16, offset=o + 16 * j))
        assert np.array_equal(y[o + 16 * j:o + 16 * j + 16].cpu().numpy(), want), (m, j)
    b.close()


def test_cbc_in_place_decryption_is_rejected(A, O):
    descs, keys = mixed_messages(A, 30, 48, mode=2, decrypt=1, min_len=32)
    x, xd, _ = buffers(descs, 48)
    b = A.Batch(descs, keys, xd, xd)
    b.run()
    planned, rejected = b.query()
    assert rejected == 30 and planned == 0
    assert np.array_equal(xd.cpu().numpy(), x)


def test_partly_overlapping_messages_are_rejected(A, O):
    """In one buffer, a message whose output starts one block after its
    input is rejected; one that runs in place (CBC decryption aside) is not."""
    descs, keys = mixed_messages(A, 12, 55, min_len=64, modes=3)
    x, xd, _ = buffers(descs, 55)
    shifted = descs.copy()
    shifted["out_off"][:6] += 16
    shifted["nbytes"][:6] = np.minimum(shifted["nbytes"][:6], descs["nbytes"][:6] - 16) // 16 * 16
    cbc_in_place = (shifted["mode"] == 2) & (shifted["decrypt"] == 1)
    b = A.Batch(shifted, keys, xd, xd)
    b.run()
    planned, rejected = b.query()
    assert rejected == 6 + int(cbc_in_place[6:].sum()) and planned == 12 - rejected


def test_many_serial_cbc_messages(A, O):
    # more CBC-encrypt messages than one wave takes (64, one per lane), with
    # parallel work mixed in
    descs, keys = mixed_messages(A, 200, 49, max_len=1 << 14, min_len=16)
    descs["mode"][:150] = 2
    descs["decrypt"][:150] = 0
    descs["nbytes"][:150] = descs["nbytes"][:150] // 16 * 16     # whole blocks (was CTR for some)
    x, xd, yd = buffers(descs, 49)
    b = A.Batch(descs, keys, xd, yd)
    b.run()
    planned, rejected = b.query()
    assert rejected == 0
    check_against_oracle(O, descs, keys, x, yd.cpu().numpy())


def test_serial_list_beyond_the_static_chunks(A, O):
    """More CBC-encrypt messages than 64 per wave of the largest grid
    (4,096 waves), so the rest are handed out from the counter: one-block
    messages under one key with their own IVs, C = Cipher(P xor IV), checked
    in one oracle ECB pass."""
    n = 64 * 4096 + 7000
    rng = np.random.default_rng(50)
    ivs = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    keys = np.zeros((1, 32), np.uint8)
    keys[0, :16] = seedgen.key(50, 0, 128)
    descs = A.make_descs(np.full(n, 16), key_idx=0, keybits=128, mode="cbc", ctr0=ivs)
    x, xd, yd = buffers(descs, 50)
    b = A.Batch(descs, keys, xd, yd)
    b.run()
    assert b.query() == (n, 0)
    rk, nr = O.expand_key(keys[0][:16])
    want = O.ecb_encrypt(rk, nr, (x[:16 * n].reshape(n, 16) ^ ivs).reshape(-1))
    assert np.array_equal(yd.cpu().numpy()[:16 * n], want)
    b.close()


@pytest.mark.parametrize("decrypt", [0, 1])
def test_xts_sector_batch_equals_plain(A, O, decrypt):
    """A storage-like batch: 3,000 requests of 1 .. 64 data units of 512 B or
    4 KiB, each with its own key pair and starting sector, against one
    aes_xts_* call per request, and sampled requests against the oracle."""
    rng = np.random.default_rng(48 + decrypt)
    n = 3000
    unit = rng.choice([512, 4096], n)
    lens = unit * rng.integers(1, 65, n)
    keybits = rng.choice([128, 256], n)
    first = rng.integers(0, 1 << 40, n)
    keys = np.zeros((2 * n, 32), np.uint8)
    ctr0 = np.zeros((n, 16), np.uint8)
    for m in range(n):
        keys[2 * m, :keybits[m] // 8] = seedgen.key(48, 2 * m, int(keybits[m]))
        keys[2 * m + 1, :keybits[m] // 8] = seedgen.key(48, 2 * m + 1, int(keybits[m]))
        ctr0[m] = A.xts_ctr0(int(first[m]), 2 * m + 1, int(unit[m]))
    descs = A.make_descs(lens, key_idx=2 * np.arange(n), keybits=keybits, mode="xts", decrypt=decrypt,
                         ctr0=ctr0)
    x, xd, yd = buffers(descs, 48)
    b = A.Batch(descs, keys, xd, yd)
    b.run()
    assert b.query()[1] == 0
    zd = torch.full_like(yd, SENTINEL)
    fn = A.aes_xts_decrypt if decrypt else A.aes_xts_encrypt
    for m in range(n):
        o, ln, bits = int(descs["in_off"][m]), int(lens[m]), int(keybits[m])
        rk1, nr = A.aes_expand_key(keys[2 * m][:bits // 8])
        rk2, _ = A.aes_expand_key(keys[2 * m + 1][:bits // 8])
        fn(xd[o:o + ln], zd[o:o + ln], ln, rk1, rk2, nr, int(unit[m]), int(first[m]))
    torch.cuda.synchronize()
    assert torch.equal(yd, zd)
    y = yd.cpu().numpy()
    check_against_oracle(O, descs[::97], keys, x, y)


def test_sector_batch_full_size_sampled(A, O):
    """The 4 KiB sector workload at its full size and in the graph launch
    the benchmark times: 65,536 messages, each with its own AES-128 key and
    IV (XTS: its own key pair, one 4 KiB data unit).  CBC encryption and XTS
    encryption are compared with the oracle on 128 sampled messages; CBC
    decryption of the whole CBC output must give back the input."""
    nmsg, size = 65536, 4096
    rng = np.random.default_rng(6)
    keys = np.zeros((2 * nmsg, 32), np.uint8)
    keys[:, :16] = rng.integers(0, 256, (2 * nmsg, 16), dtype=np.uint8)
    ivs = rng.integers(0, 256, (nmsg, 16), dtype=np.uint8)
    xts = np.stack([A.xts_ctr0(m, nmsg + m, size) for m in range(nmsg)])
    x = seedgen.data_torch(6, 0, nmsg * size, "cuda")
    idx = np.sort(np.random.default_rng(61).choice(nmsg, 128, replace=False))
    rows = torch.from_numpy(idx).cuda()
    xs = x.view(nmsg, size)[rows].cpu().numpy()

    def run(descs, src):
        out = torch.full_like(src, SENTINEL)
        b = A.Batch(descs, keys, src, out)
        b.launch_graph()
        torch.cuda.synchronize()
        assert b.query() == (nmsg, 0)
        b.close()
        return out

    cbc = A.make_descs(np.full(nmsg, size), keybits=128, mode="cbc", decrypt=0, ctr0=ivs)
    y = run(cbc, x)
    ys = y.view(nmsg, size)[rows].cpu().numpy()
    for j, m in enumerate(idx):
        assert np.array_equal(ys[j], oracle_message(O, cbc[m], keys, xs[j])), ("CBC encrypt", m)
    z = run(A.make_descs(np.full(nmsg, size), keybits=128, mode="cbc", decrypt=1, ctr0=ivs), y)
    assert torch.equal(z, x)
    del z
    xd = A.make_descs(np.full(nmsg, size), keybits=128, mode="xts", decrypt=0, ctr0=xts)
    w = run(xd, x)
    ws = w.view(nmsg, size)[rows].cpu().numpy()
    for j, m in enumerate(idx):
        assert np.array_equal(ws[j], oracle_message(O, xd[m], keys, xs[j])), ("XTS encrypt", m)


# --- GCM messages in a batch -------------------------------------------------
def gcm_batch(A, O, n, seed, max_len=1 << 16, big=(), n_other=0, big_aad=None, big_bits=None):
    """n GCM messages (and n_other CTR/ECB ones), 128/192/256-bit keys,
    lengths log-uniform up to max_len plus the lengths in `big`, additional
    data of 0 .. 1000 bytes (larger for the big ones), half encryptions and
    half decryptions of the oracle's ciphertexts, a quarter of those with a
    changed tag.  Input buffer: the messages, then their additional data,
    then the expected tags; output buffer: the same size (tags of the
    encryptions at the same offsets as the expected tags)."""
    rng = np.random.default_rng(seed)
    lens = list(seedgen.log_uniform_lengths(rng, n, 1, max_len)) + list(big)
    n = len(lens)
    lens[0] = 0
    keybits = rng.choice([128, 192, 256], n + n_other)
    if big_bits is not None:
        keybits[n - len(big):n] = big_bits
    dec = rng.integers(0, 2, n)
    aadl = rng.integers(0, 1001, n)
    aadl[1] = 0
    for i in range(len(big)):
        aadl[n - len(big) + i] = big_aad[i] if big_aad is not None else 100000 + 7 * (len(big) - 1 - i)
    keys = np.zeros((n + n_other, 32), np.uint8)
    for m in range(n + n_other):
        keys[m, :keybits[m] // 8] = seedgen.key(seed, m, int(keybits[m]))
    ivs = [seedgen.nonce(seed, m)[:12] for m in range(n)]
    olens = seedgen.log_uniform_lengths(rng, n_other, 16, max_len, 16) if n_other else np.zeros(0, np.int64)
    pad = lambda v: (int(v) + 15) // 16 * 16  # noqa: E731
    off, msg_off = 0, []
    for L in list(lens) + list(olens):
        msg_off.append(off)
        off += pad(L)
    aad_off = []
    for L in aadl:
        aad_off.append(off)
        off += pad(L)
    tag_off = []
    for _ in range(n):
        tag_off.append(off)
        off += 16
    total = off + 16
    x = np.zeros(total, np.uint8)
    want = {}
    forged = np.zeros(n, bool)
    for m in range(n):
        bits = int(keybits[m])
        rk, nr = O.expand_key(keys[m][:bits // 8])
        pt = seedgen.data_np(seed, 1000 + m, int(lens[m]))
        aad = seedgen.data_np(seed, 5000 + m, int(aadl[m]))
        ct, tag = O.gcm_encrypt(rk, nr, ivs[m], aad, pt)
        x[aad_off[m]:aad_off[m] + aad.size] = aad
        if dec[m]:
            x[msg_off[m]:msg_off[m] + ct.size] = ct
            t = tag.copy()
            if m % 4 == 1:
                t[m % 16] ^= 0x40
                forged[m] = True
            x[tag_off[m]:tag_off[m] + 16] = t
            want[m] = (pt, None, not forged[m])
        else:
            x[msg_off[m]:msg_off[m] + pt.size] = pt
            want[m] = (ct, tag, True)
    for k in range(n_other):
        m = n + k
        x[msg_off[m]:msg_off[m] + int(olens[k])] = seedgen.data_np(seed, 9000 + k, int(olens[k]))
    modes = [A.AES_MODE_GCM] * n + [int(v) for v in rng.choice([0, 1], n_other)]
    ctr0 = np.zeros((n + n_other, 16), np.uint8)
    for m in range(n):
        ctr0[m, :12] = ivs[m]
    for k in range(n_other):
        ctr0[n + k] = seedgen.nonce(seed, n + k)
    descs = A.make_descs(list(lens) + list(olens), in_off=msg_off, keybits=keybits, mode=modes,
                         decrypt=list(dec) + [0] * n_other, ctr0=ctr0)
    g = np.zeros(n + n_other, A.GCM_DESC_DTYPE)
    g["aad_off"][:n] = aad_off
    g["aad_bytes"][:n] = aadl
    g["tag_off"][:n] = tag_off
    g["tag_bytes"][:n] = 16
    g["ok"] = -7
    return descs, keys, g, x, want, n


def check_gcm_batch(A, O, b, descs, keys, x, y, want, n, g_out):
    for m in range(n):
        d = descs[m]
        o, L = int(d["out_off"]), int(d["nbytes"])
        data, tag, ok = want[m]
        assert np.array_equal(y[o:o + L], data), "GCM message %d (%s) output" % (m, d)
        if tag is not None:
            t = int(g_out["tag_off"][m])
            assert np.array_equal(y[t:t + 16], tag), "GCM message %d tag" % m
        assert g_out["ok"][m] == (1 if ok else 0), "GCM message %d verdict" % m
    # the other messages, against the oracle
    for m in range(n, len(descs)):
        d = descs[m]
        i, L = int(d["in_off"]), int(d["nbytes"])
        want_o = oracle_message(O, d, keys, x[i:i + L])
        assert np.array_equal(y[int(d["out_off"]):int(d["out_off"]) + L], want_o), "message %d" % m


def test_gcm_batch_matches_oracle(A, O):
    descs, keys, g, x, want, n = gcm_batch(A, O, 200, 71, big=((1 << 20) + 5, 600 * 1024 + 3), n_other=40)
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.zeros_like(xd)
    b = A.Batch(descs, keys, xd, yd, gcm=g)
    b.run()
    planned, rejected = b.query()
    assert rejected == 0 and planned == len(descs)
    check_gcm_batch(A, O, b, descs, keys, x, yd.cpu().numpy(), want, n, b.gcm_results(len(descs)))
    # graph replays recompute everything from the descriptors (the sums start over)
    yd.zero_()
    b.launch_graph()
    b.launch_graph()
    torch.cuda.synchronize()
    check_gcm_batch(A, O, b, descs, keys, x, yd.cpu().numpy(), want, n, b.gcm_results(len(descs)))
    b.close()


def test_gcm_batch_refuses_bad_fields(A, O):
    descs, keys, g, x, want, n = gcm_batch(A, O, 8, 72)
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.zeros_like(xd)
    bad = g.copy()
    bad["aad_off"][2] += 8                                      # not 16-byte aligned
    bad["aad_bytes"][3] = xd.numel()                            # past the input buffer
    bad["tag_off"][4] = xd.numel() - 8                          # the tag past the buffer's end
    if descs["decrypt"][5]:
        bad["tag_bytes"][5] = 7                                 # a tag length the standard does not allow
    else:
        bad["tag_off"][5] = int(descs["out_off"][5])            # the tag over the message's own output
    b = A.Batch(descs, keys, xd, yd, gcm=bad)
    b.run()
    _, rejected = b.query()
    assert rejected == 4
    r = b.gcm_results(len(descs))
    assert list(r["ok"][2:6]) == [0, 0, 0, 0]
    check_gcm_batch(A, O, b, descs[6:], keys[6:], x, yd.cpu().numpy(), {i - 6: want[i] for i in range(6, n)},
                    n - 6, r[6:])
    # without GCM fields every GCM descriptor is refused
    b2 = A.Batch(descs, keys, xd, yd)
    b2.run()
    assert b2.query()[1] == n


def test_gcm_batch_piece_boundaries(A, O):
    """Messages around the edges of the GHASH pieces of 4,096 positions
    (position 0 the length block, 1 .. nC the ciphertext blocks from the
    last, then the additional data): a piece made only of whole ciphertext
    blocks takes the hash's fast path, here with its last position exactly
    the first ciphertext block (nC = 8,191 and 12,287), one short of it,
    with and without a partial last block and additional data."""
    big, big_aad = [], []
    for nc in (4095, 4096, 4097, 8190, 8191, 8192, 12287):
        for t, aad in ((0, 0), (1, 0), (15, 33), (0, 16)):
            big.append(16 * nc - t)
            big_aad.append(aad)
    descs, keys, g, x, want, n = gcm_batch(A, O, 3, 79, max_len=64, big=big, big_aad=big_aad)
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.zeros_like(xd)
    b = A.Batch(descs, keys, xd, yd, gcm=g)
    b.run()
    assert b.query() == (len(descs), 0)
    check_gcm_batch(A, O, b, descs, keys, x, yd.cpu().numpy(), want, n, b.gcm_results(len(descs)))
    b.close()


def test_gcm_batch_fused_messages(A, O):
    """GCM messages of at least 2 x 65,536 GHASH positions (about 2 MiB) are
    encrypted and hashed in one pass, one workgroup per piece of 65,536
    positions: messages at the threshold and one short of it, partial last
    blocks, additional data long enough to fill slow steps, every key size,
    both directions and forged tags, beside short GCM messages and other
    modes in the same batch, against the oracle; then a graph replay."""
    K = 65536
    big = [16 * (2 * K - 1), 16 * (2 * K - 1) - 1, 16 * (2 * K - 2), 16 * (3 * K) + 5, 16 * (2 * K + 37) + 9,
           16 * (2 * K) + 1]
    big_aad = [0, 0, 0, 16 * 100 + 3, 70000, 17]
    big_bits = [128, 192, 256, 256, 128, 192]
    descs, keys, g, x, want, n = gcm_batch(A, O, 30, 83, max_len=1 << 14, big=big, n_other=12, big_aad=big_aad,
                                           big_bits=big_bits)
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.zeros_like(xd)
    b = A.Batch(descs, keys, xd, yd, gcm=g)
    b.run()
    assert b.query() == (len(descs), 0)
    check_gcm_batch(A, O, b, descs, keys, x, yd.cpu().numpy(), want, n, b.gcm_results(len(descs)))
    yd.zero_()
    b.launch_graph()
    b.launch_graph()
    torch.cuda.synchronize()
    check_gcm_batch(A, O, b, descs, keys, x, yd.cpu().numpy(), want, n, b.gcm_results(len(descs)))
    assert b.c.gcm_two_pass == 0
    b.close()
    # the same batch with two passes for every message
    y2 = torch.zeros_like(xd)
    b2 = A.Batch(descs, keys, xd, y2, gcm=g, gcm_two_pass=True)
    assert b2.c.gcm_two_pass == 1
    b2.run()
    assert b2.query() == (len(descs), 0)
    check_gcm_batch(A, O, b2, descs, keys, x, y2.cpu().numpy(), want, n, b2.gcm_results(len(descs)))
    b2.close()


def test_gcm_batch_message_beyond_the_stored_powers(A):
    """One GCM message of 512 MiB + 80 KiB: its GHASH pieces run past the
    13 powers H^(4096 * 2^t) kept per message, so the last ones square on.
    It equals the single-buffer GCM kernels' ciphertext and tag (a separate
    implementation, checked against the oracle elsewhere, at 1 GiB through
    GHASH's linearity)."""
    n = (512 << 20) + 80 * 1024 + 7
    key = np.zeros((1, 32), np.uint8)
    key[0, :16] = seedgen.key(73, 0, 128)
    iv = seedgen.nonce(73, 0)[:12]
    x = seedgen.data_torch(73, 0, n + 64, "cuda")
    y = torch.zeros_like(x)
    aad_off = (n + 15) // 16 * 16                      # 48 bytes of additional data after the message
    descs = A.make_descs([n], in_off=[0], keybits=128, mode="gcm", ctr0=np.concatenate([iv, np.zeros(4, np.uint8)]))
    g = np.zeros(1, A.GCM_DESC_DTYPE)
    g["aad_off"], g["aad_bytes"], g["tag_off"], g["tag_bytes"] = aad_off, 48, aad_off, 16
    b = A.Batch(descs, key, x, y, gcm=g)
    b.run()
    assert b.query() == (1, 0)
    assert b.gcm_results(1)["ok"][0] == 1
    rk, nr = A.aes_expand_key(key[0, :16])
    ws = torch.zeros(A.aes_gcm_workspace_size(), dtype=torch.uint8, device="cuda")
    ref_out = torch.empty(n, dtype=torch.uint8, device="cuda")
    tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
    A.aes_gcm_encrypt(x[:n], ref_out, n, x[aad_off:aad_off + 48], 48, rk, nr, iv, tag, ws)
    torch.cuda.synchronize()
    assert torch.equal(y[:n], ref_out)
    assert torch.equal(y[aad_off:aad_off + 16], tag)
    del x, y, ref_out
    torch.cuda.empty_cache()


def _batch_header_nlane(b):
    """GCM messages the last run of batch b hashed one per lane (the
    workspace header's count: byte 72 of the 256-byte header at the
    workspace's 256-byte aligned start)."""
    off = (b.workspace.data_ptr() + 255) // 256 * 256 - b.workspace.data_ptr()
    hdr = b.workspace[off:off + 256].cpu().numpy()
    return int(hdr[72:76].view(np.uint32)[0])


def test_gcm_batch_many_short_messages_one_per_lane(A, O):
    """34,000 short GCM messages (0 .. 4 KiB, additional data 0 .. 1 KiB,
    AES-128/256): enough that the batch hashes them one per lane.  A sample
    and the size boundary (512 GHASH positions: per lane; 513: in pieces)
    against the oracle; every ciphertext and tag against the same messages
    run as two batches of 17,000, which hash in pieces; then every message
    decrypted with its tag, a quarter of the tags changed, which must be
    refused."""
    n = 34000
    rng = np.random.default_rng(81)
    lens = seedgen.log_uniform_lengths(rng, n, 1, 4096)
    lens[:3] = [0, 1, 16]
    aadl = rng.integers(0, 1025, n)
    aadl[:3] = [0, 0, 1]
    # GHASH positions = ceil(aad/16) + ceil(len/16) + 1: 512 and 513
    lens[3], aadl[3] = 4096, 255 * 16          # 255 + 256 + 1 = 512
    lens[4], aadl[4] = 4095, 255 * 16 + 1      # 256 + 256 + 1 = 513
    keybits = rng.choice([128, 256], n)
    pad = (lens + 15) // 16 * 16
    msg_off = np.concatenate([[0], np.cumsum(pad)[:-1]])
    aad_base = int(pad.sum())
    apad = (aadl + 15) // 16 * 16
    aad_off = aad_base + np.concatenate([[0], np.cumsum(apad)[:-1]])
    tag_base = aad_base + int(apad.sum())
    tag_off = tag_base + 16 * np.arange(n)
    total = tag_base + 16 * n + 16
    x = rng.integers(0, 256, total, dtype=np.uint8)
    keys = np.zeros((n, 32), np.uint8)
    keys[:, :32] = rng.integers(0, 256, (n, 32), dtype=np.uint8)
    keys[keybits == 128, 16:] = 0
    ctr0 = np.zeros((n, 16), np.uint8)
    ctr0[:, :12] = rng.integers(0, 256, (n, 12), dtype=np.uint8)
    g = np.zeros(n, A.GCM_DESC_DTYPE)
    g["aad_off"], g["aad_bytes"], g["tag_off"], g["tag_bytes"] = aad_off, aadl, tag_off, 16
    enc = A.make_descs(lens, in_off=msg_off, keybits=keybits, mode="gcm", ctr0=ctr0)

    xd = torch.from_numpy(x).to("cuda")
    yd = torch.zeros_like(xd)
    b = A.Batch(enc, keys, xd, yd, gcm=g)
    b.run()
    assert b.query() == (n, 0)
    assert _batch_header_nlane(b) == n - 1           # all but the 513-position message
    r = b.gcm_results(n)
    assert (r["ok"] == 1).all()
    y = yd.cpu().numpy()
    # replays of the captured graph give the same bytes (the plan, the lists
    # and the sums start over at every launch)
    for _ in range(2):
        yd.zero_()
        b.launch_graph()
        torch.cuda.synchronize()
        assert np.array_equal(yd.cpu().numpy(), y)
    b.close()

    # the oracle on a sample and on the boundary messages
    for m in sorted(set(rng.choice(n, 300, replace=False).tolist()) | {0, 1, 2, 3, 4}):
        bits = int(keybits[m])
        rk, nr = O.expand_key(keys[m, :bits // 8])
        pt = x[msg_off[m]:msg_off[m] + lens[m]]
        aad = x[aad_off[m]:aad_off[m] + aadl[m]]
        ct, tag = O.gcm_encrypt(rk, nr, ctr0[m, :12], aad, pt)
        assert np.array_equal(y[msg_off[m]:msg_off[m] + lens[m]], ct), ("ciphertext", m)
        assert np.array_equal(y[tag_off[m]:tag_off[m] + 16], tag), ("tag", m)

    # the same messages as two batches below the per-lane threshold: GHASH in pieces
    y2 = torch.zeros_like(xd)
    half = n // 2
    for lo, hi in ((0, half), (half, n)):
        bh = A.Batch(enc[lo:hi], keys, xd, y2, gcm=g[lo:hi])
        bh.run()
        assert bh.query() == (hi - lo, 0)
        assert _batch_header_nlane(bh) == 0
        bh.close()
    assert np.array_equal(y2.cpu().numpy()[:tag_base + 16 * n], y[:tag_base + 16 * n])

    # decryption of every message with its tag; a quarter of the tags changed
    xin = y.copy()
    xin[aad_base:tag_base] = x[aad_base:tag_base]     # the additional data
    forged = np.arange(n) % 4 == 1
    xin[tag_off[forged] + (np.arange(n)[forged] % 16)] ^= 0x20
    dec = enc.copy()
    dec["decrypt"] = 1
    xd2 = torch.from_numpy(xin).to("cuda")
    zd = torch.zeros_like(xd2)
    g["ok"] = -7
    bd = A.Batch(dec, keys, xd2, zd, gcm=g)
    bd.run()
    assert bd.query() == (n, 0)
    assert _batch_header_nlane(bd) == n - 1
    rd = bd.gcm_results(n)
    assert np.array_equal(rd["ok"], np.where(forged, 0, 1).astype(rd["ok"].dtype))
    # every plaintext recovered (the output holds it whatever the verdict);
    # the padding between messages untouched
    z = zd.cpu().numpy()[:aad_base]
    inside = np.repeat(np.tile([True, False], n), np.column_stack([lens, pad - lens]).ravel())
    assert np.array_equal(z[inside], x[:aad_base][inside])
    assert not z[~inside].any()
    bd.close()
    del xd, yd, y2, xd2, zd
    torch.cuda.empty_cache()


def _gcm_random_batch(A, seed, lens, aad_lens, base=0):
    """GCM descriptors over random data: messages back to back from `base`,
    then their additional data, then one 16-byte tag slot each (random bytes:
    the expected tags of the decryptions); encryptions and decryptions, key
    sizes and IVs at random."""
    rng = np.random.default_rng(seed)
    n = len(lens)
    pad = lambda v: (int(v) + 15) // 16 * 16  # noqa: E731
    off, msg_off, aad_off, tag_off = base, [], [], []
    for L in lens:
        msg_off.append(off)
        off += pad(L)
    for L in aad_lens:
        aad_off.append(off)
        off += pad(L)
    for _ in range(n):
        tag_off.append(off)
        off += 16
    keybits = rng.choice([128, 192, 256], n)
    keys = np.zeros((n, 32), np.uint8)
    keys[:, :] = rng.integers(0, 256, (n, 32), dtype=np.uint8)
    ctr0 = np.zeros((n, 16), np.uint8)
    ctr0[:, :12] = rng.integers(0, 256, (n, 12), dtype=np.uint8)
    descs = A.make_descs(list(lens), in_off=msg_off, keybits=keybits, mode="gcm",
                         decrypt=list(rng.integers(0, 2, n)), ctr0=ctr0)
    g = np.zeros(n, A.GCM_DESC_DTYPE)
    g["aad_off"], g["aad_bytes"], g["tag_off"], g["tag_bytes"] = aad_off, aad_lens, tag_off, 16
    return descs, keys, g, off


def _gcm_results(yd, descs, g):
    """Outputs, encryption tags and verdicts of a finished GCM batch."""
    y = yd.cpu().numpy()
    outs = [y[int(d["out_off"]):int(d["out_off"]) + int(d["nbytes"])] for d in descs]
    tags = [y[int(t):int(t) + 16] if not d["decrypt"] else None for d, t in zip(descs, g["tag_off"])]
    return outs, tags


def test_gcm_batch_one_pass_in_place_and_replayed(A):
    """The one-pass kernels in place (output over input) and from a graph
    replayed with rewritten descriptors equal the two-pass kernels on the
    same messages: outputs, tags and verdicts (the two-pass path is checked
    against the oracle elsewhere)."""
    K = 65536
    lens = [16 * (2 * K) + 5, 16 * (3 * K) - 1, 16 * (2 * K + 300), 0, 17, 4096, 100000, 16 * (5 * K) + 8]
    aad_lens = [0, 33, 16 * 700, 5, 0, 64, 1000, 0]
    descs, keys, g, total = _gcm_random_batch(A, 91, lens, aad_lens)
    x = torch.randint(0, 256, (total + 64,), dtype=torch.uint8, device="cuda")

    def run(descs, keys, g, two_pass, inplace, graph=None):
        src = x.clone()
        dst = src if inplace else torch.zeros_like(x)
        b = A.Batch(descs, keys, src, dst, gcm=g, gcm_two_pass=two_pass)
        b.run()
        torch.cuda.synchronize()
        assert b.query() == (len(descs), 0)
        res = _gcm_results(dst, descs, g), b.gcm_results(len(descs))["ok"].copy()
        b.close()
        return res

    (want_o, want_t), want_ok = run(descs, keys, g, True, False)
    (got_o, got_t), got_ok = run(descs, keys, g, False, True)
    assert list(got_ok) == list(want_ok)
    for m in range(len(descs)):
        assert np.array_equal(got_o[m], want_o[m]), "message %d in place" % m
        if want_t[m] is not None:
            assert np.array_equal(got_t[m], want_t[m]), "message %d tag in place" % m
    # a graph with room for 12 messages, replayed with rewritten descriptors
    y = torch.zeros_like(x)
    b = A.Batch(descs, keys, x, y, gcm=g, max_msgs=12, gcm_two_pass=False)
    b.launch_graph()
    torch.cuda.synchronize()
    (o1, t1) = _gcm_results(y, descs, g)
    for m in range(len(descs)):
        assert np.array_equal(o1[m], want_o[m]), "message %d from the graph" % m
        if want_t[m] is not None:
            assert np.array_equal(t1[m], want_t[m]), "message %d tag from the graph" % m
    lens2 = [16 * (4 * K) + 3, 50, 16 * (2 * K) - 16, 16 * (2 * K) + 1, 7000]
    descs2, keys2, g2, total2 = _gcm_random_batch(A, 92, lens2, [0, 16, 48, 0, 3])
    assert total2 <= total
    (want2_o, want2_t), want2_ok = run(descs2, keys2, g2, True, False)
    y.zero_()
    b.set_descs(descs2, keys2, gcm=g2)
    b.launch_graph()
    torch.cuda.synchronize()
    (o2, t2) = _gcm_results(y, descs2, g2)
    assert list(b.gcm_results(len(descs2))["ok"]) == list(want2_ok)
    for m in range(len(descs2)):
        assert np.array_equal(o2[m], want2_o[m]), "rewritten message %d from the graph" % m
        if want2_t[m] is not None:
            assert np.array_equal(t2[m], want2_t[m]), "rewritten message %d tag from the graph" % m
    b.close()
