"""The batch call that allocates nothing (aes_batch_run_noalloc: the
library's own device-resident workspace instead of the caller's), through
the C ABI, against the existing batch call (aes_batch_run with a caller
workspace) on the same messages, bit for bit: two calls in a row, the second
with a smaller batch, so the second runs on what the first left behind."""
import ctypes

import numpy as np
import pytest

import seedgen
from oracle import ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SENTINEL = 0x5A


@pytest.fixture(scope="module")
def A():
    from paper_1403_7295_amd import aesgpu
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return aesgpu


def messages(A, n, seed, max_len):
    """n messages of every mode and direction (ECB, CTR, CBC, XTS), 128/192/
    256-bit keys, lengths log-uniform up to max_len (whole blocks except
    CTR), packed back to back."""
    rng = np.random.default_rng(seed)
    lens = seedgen.log_uniform_lengths(rng, n, 1, max_len)
    mode = rng.integers(0, 4, n)
    decrypt = rng.integers(0, 2, n)
    keybits = rng.choice([128, 192, 256], n)
    lens = np.where(mode != 1, (lens + 15) // 16 * 16, lens)
    keys = np.zeros((n, 32), np.uint8)
    ctr0 = np.zeros((n, 16), np.uint8)
    units = rng.choice([16, 512, 4096], n)
    for m in range(n):
        keys[m, :keybits[m] // 8] = seedgen.key(seed, m, int(keybits[m]))
        ctr0[m] = seedgen.nonce(seed, m)
        if mode[m] == 3:
            ctr0[m] = A.xts_ctr0(int(rng.integers(0, 1 << 62)), (m + 1) % n, int(units[m]))
    return A.make_descs(lens, keybits=keybits, mode=mode, decrypt=decrypt, ctr0=ctr0), keys


def run_both(A, descs, keys, seed):
    """The same batch through aes_batch_run (caller workspace) and through
    aes_batch_run_noalloc, each into its own sentinel-filled output."""
    end = int((descs["in_off"] + descs["nbytes"]).max())
    total = (end + 15) // 16 * 16 + 16
    xd = seedgen.data_torch(seed, 7, total, "cuda")
    y_ref = torch.full_like(xd, SENTINEL)
    y_na = torch.full_like(xd, SENTINEL)
    b = A.Batch(descs, keys, xd, y_ref)
    b.run()
    planned, rejected = b.query()
    assert rejected == 0 and planned == len(descs)
    c = A.aes_batch.from_buffer_copy(b.c)
    c.out_base = y_na.data_ptr()
    c.workspace = None
    c.workspace_bytes = 0
    stream = torch.cuda.current_stream().cuda_stream
    rc = A.lib.aes_batch_run_noalloc(ctypes.byref(c), ctypes.c_void_p(stream))
    assert rc == A.AES_OK, A.aes_last_error()
    torch.cuda.synchronize()
    return xd, y_ref, y_na


def test_noalloc_equals_batch_run_twice_second_smaller(A):
    o = ref.default()
    first, keys1 = messages(A, 3000, 61, 1 << 18)
    second, keys2 = messages(A, 700, 62, 1 << 14)
    assert len(second) < len(first) and second["nbytes"].sum() < first["nbytes"].sum()
    for descs, keys, seed in ((first, keys1, 61), (second, keys2, 62)):
        xd, y_ref, y_na = run_both(A, descs, keys, seed)
        assert torch.equal(y_na, y_ref), "%d messages" % len(descs)
        # and a few messages of each call against the oracle
        x, y = xd.cpu().numpy(), y_na.cpu().numpy()
        for m in range(0, len(descs), max(1, len(descs) // 8)):
            d = descs[m]
            n, i = int(d["nbytes"]), int(d["in_off"])
            bits = 128 + 64 * int(d["keybits_code"])
            rk, nr = o.expand_key(keys[m][:bits // 8])
            if d["mode"] == 1:
                want = o.ctr(rk, nr, d["ctr0"], x[i:i + n])
            elif d["mode"] == 0:
                want = o.ecb(bool(d["decrypt"]), rk, nr, x[i:i + n])
            else:
                continue
            assert np.array_equal(y[i:i + n], want), "message %d" % m


def test_noalloc_graph_count_from_device(A):
    # the message count read from the device (d_nmsg), as a captured caller does
    descs, keys = messages(A, 400, 63, 1 << 16)
    xd, y_ref, _ = run_both(A, descs, keys, 63)
    y_na = torch.full_like(xd, SENTINEL)
    b = A.Batch(descs, keys, xd, y_ref)
    c = A.aes_batch.from_buffer_copy(b.c)
    c.out_base = y_na.data_ptr()
    c.workspace = None
    c.workspace_bytes = 0
    c.d_nmsg = b.d_nmsg.data_ptr()
    c.nmsg = 0
    A.aes_batch_run_noalloc(c)
    torch.cuda.synchronize()
    assert torch.equal(y_na, y_ref)
