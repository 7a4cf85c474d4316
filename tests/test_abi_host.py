"""The C-ABI library on the CPU: it loads, exports every function its header
declares, and its host-side logic (key schedule, argument checks) behaves as
documented.  Nothing here launches a kernel: every call below returns before
the library touches a device."""
import os
import re
import subprocess

import numpy as np
import pytest

import seedgen
from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aesgpu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aes_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def A():
    from paper_1403_7295_amd import aesgpu
    return aesgpu


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("aes_expand_key", "aes_encrypt", "aes_decrypt", "aes_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(A):
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (aes_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(declared_functions()) == set(A._SIGNATURES)


@pytest.mark.parametrize("bits", [128, 192, 256])
def test_key_schedule_matches_oracle(A, bits):
    o = ref.default()
    for i in range(16):
        k = seedgen.key(77, 100 * bits + i, bits)
        rk, nr = A.aes_expand_key(k)
        rk_ref, nr_ref = o.expand_key(k)
        assert nr == nr_ref == bits // 32 + 6
        assert np.array_equal(rk, rk_ref)


def test_bad_key_size(A):
    with pytest.raises(A.AESError) as e:
        A.aes_expand_key(np.zeros(20, np.uint8), 160)
    assert e.value.code == A.AES_E_KEYBITS


# Fake, never-dereferenced device addresses: every case below is rejected (or
# is a no-op) before the library looks at a device.
IN, OUT = 0x10000, 0x20000


@pytest.mark.parametrize("fn", ["aes_encrypt", "aes_decrypt"])
def test_argument_checks(A, fn):
    rk, nr = A.aes_expand_key(np.zeros(16, np.uint8))
    call = getattr(A, fn)

    def code(*args, **kw):
        with pytest.raises(A.AESError) as e:
            call(*args, stream=0, **kw)
        return e.value.code

    assert code(IN, OUT, 32, rk, 11, "ecb") == A.AES_E_NR
    assert code(IN, OUT, 32, rk, nr, 5) == A.AES_E_MODE
    assert code(IN, OUT, 32, rk, nr, "cbc") == A.AES_E_NULL         # no IV
    assert code(IN, OUT, 24, rk, nr, "cbc", ctr0=bytes(16)) == A.AES_E_LENGTH
    assert code(IN, OUT, 17, rk, nr, "ecb") == A.AES_E_LENGTH
    assert code(IN, OUT, 32, rk, nr, "ctr") == A.AES_E_NULL          # no counter block
    assert code(None, OUT, 32, rk, nr, "ecb") == A.AES_E_NULL
    assert code(IN + 4, OUT, 32, rk, nr, "ecb") == A.AES_E_ALIGN
    assert code(IN, IN + 16, 64, rk, nr, "ecb") == A.AES_E_OVERLAP
    assert code(IN + 16, IN, 64, rk, nr, "ctr", ctr0=bytes(16)) == A.AES_E_OVERLAP
    if fn == "aes_decrypt":
        assert code(IN, IN, 64, rk, nr, "cbc", ctr0=bytes(16)) == A.AES_E_OVERLAP   # not in place
    # CTR: at most 2^32 blocks per call (the 32-bit counter must not repeat)
    assert code(IN, OUT, (1 << 36) + 1, rk, nr, "ctr", ctr0=bytes(16)) == A.AES_E_LENGTH
    # empty buffers are a no-op, whatever the pointers
    call(None, None, 0, rk, nr, "ecb", stream=0)
    call(None, None, 0, rk, nr, "ctr", ctr0=bytes(16), stream=0)


@pytest.mark.parametrize("fn", ["aes_xts_encrypt", "aes_xts_decrypt"])
def test_xts_argument_checks(A, fn):
    rk, nr = A.aes_expand_key(np.zeros(32, np.uint8))
    call = getattr(A, fn)

    def code(*args, **kw):
        with pytest.raises(A.AESError) as e:
            call(*args, stream=0, **kw)
        return e.value.code

    assert code(IN, OUT, 512, rk, rk, 11, 512) == A.AES_E_NR
    assert code(IN, OUT, 512, None, rk, nr, 512) == A.AES_E_NULL
    assert code(IN, OUT, 512, rk, None, nr, 512) == A.AES_E_NULL
    for unit in (0, 8, 48, 520, 8192):
        assert code(IN, OUT, 512, rk, rk, nr, unit) == A.AES_E_ARG
    assert code(IN, OUT, 520, rk, rk, nr, 512) == A.AES_E_LENGTH     # no ciphertext stealing
    assert code(None, OUT, 512, rk, rk, nr, 512) == A.AES_E_NULL
    assert code(IN + 8, OUT, 512, rk, rk, nr, 512) == A.AES_E_ALIGN
    assert code(IN, IN + 16, 512, rk, rk, nr, 512) == A.AES_E_OVERLAP
    call(None, None, 0, rk, rk, nr, 4096, stream=0)                 # empty: a no-op


def test_gcm_argument_checks(A):
    rk, nr = A.aes_expand_key(np.zeros(16, np.uint8))
    WS, TAG, OK, AAD = 0x40000, 0x50000, 0x60000, 0x70000
    wsb = A.aes_gcm_workspace_size()
    assert wsb >= 4096

    def enc(*args, **kw):
        f = dict(inp=IN, out=OUT, nbytes=64, aad=AAD, aad_bytes=16, roundkeys=rk, Nr=nr, iv=bytes(12),
                 tag=TAG, workspace=WS, workspace_bytes=wsb, stream=0)
        f.update(kw)
        with pytest.raises(A.AESError) as e:
            A.aes_gcm_encrypt(**f)
        return e.value.code

    def dec(**kw):
        f = dict(inp=IN, out=OUT, nbytes=64, aad=AAD, aad_bytes=16, roundkeys=rk, Nr=nr, iv=bytes(12),
                 tag=TAG, tag_bytes=16, ok=OK, workspace=WS, workspace_bytes=wsb, stream=0)
        f.update(kw)
        with pytest.raises(A.AESError) as e:
            A.aes_gcm_decrypt(**f)
        return e.value.code

    assert enc(Nr=11) == A.AES_E_NR
    assert enc(tag=None) == A.AES_E_NULL
    assert enc(workspace=None) == A.AES_E_NULL
    assert enc(iv=b"") == A.AES_E_NULL or enc(iv=b"") == A.AES_E_ARG
    assert enc(iv=bytes(257)) == A.AES_E_ARG
    assert enc(aad=None) == A.AES_E_NULL
    assert enc(aad=AAD + 8) == A.AES_E_ALIGN
    assert enc(workspace=WS + 16) == A.AES_E_ALIGN
    assert enc(workspace_bytes=wsb - 1) == A.AES_E_LENGTH
    assert enc(nbytes=(1 << 36)) == A.AES_E_LENGTH
    assert enc(inp=IN + 4) == A.AES_E_ALIGN
    assert enc(out=IN + 16) == A.AES_E_OVERLAP
    assert enc(aad=OUT + 16, aad_bytes=16) == A.AES_E_OVERLAP
    assert dec(ok=None) == A.AES_E_NULL
    for tb in (0, 3, 5, 9, 11, 17):
        assert dec(tag_bytes=tb) == A.AES_E_ARG


def test_launch_config_validation(A):
    for bad in ({"layout": 5}, {"layout": -1}, {"blocks_per_thread": 3}, {"wg_size": 100}, {"grid": -1}):
        with pytest.raises(A.AESError) as e:
            A.aes_set_launch(bad)
        assert e.value.code == A.AES_E_ARG
    for layout in (0, 1, 2, 3, 4):
        A.aes_set_launch({"layout": layout, "blocks_per_thread": 4, "wg_size": 512, "grid": 3})
    A.aes_set_launch(None)


def test_batch_workspace_size(A):
    # header + key slots of 512 bytes + five lists of 16-byte items (forward,
    # inverse, serial, GHASH, fused GCM) + the plan's fifteen 8-byte counters
    # per chunk of 256 messages
    assert A.aes_batch_workspace_size(10) == 256 + 10 * 512 + 5 * 10 * 16 + 120
    assert A.aes_batch_workspace_size(1) == 256 + 512 + 5 * 16 + 120
    assert A.aes_batch_workspace_size(257) == 256 + 257 * 512 + 5 * 257 * 16 + 2 * 120
    for bad in (0, -3):
        with pytest.raises(A.AESError) as e:
            A.aes_batch_workspace_size(bad)
        assert e.value.code == A.AES_E_ARG


def test_batch_plan_is_the_workspace_size(A):
    for n in (1, 10, 256, 257, 10000):
        assert A.aes_batch_plan(n) == A.aes_batch_workspace_size(n)
        assert A.aes_batch_plan(n, d_desc=0x100000) == A.aes_batch_workspace_size(n)
    with pytest.raises(A.AESError) as e:
        A.aes_batch_plan(0)
    assert e.value.code == A.AES_E_ARG


def test_status_codes_match_the_header(A):
    text = open(HEADER).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"\b(AES_E_[A-Z]+|AES_OK) = (\d+)", text))
    assert len(codes) == 11
    for k, v in codes.items():
        assert getattr(A, k) == v, k


def test_batch_argument_checks(A):
    ws = A.aes_batch_workspace_size(4)

    def batch(**kw):
        f = dict(desc=0x100000, nmsg=4, d_nmsg=None, keys=0x200000, nkeys=4,
                 in_base=0x300000, in_bytes=4096, out_base=0x400000, out_bytes=4096,
                 workspace=0x500000, workspace_bytes=ws, max_msgs=4, tile_blocks=0)
        f.update(kw)
        return A.aes_batch(**f)

    def code(b):
        with pytest.raises(A.AESError) as e:
            A.aes_batch_run(b, stream=0)
        return e.value.code

    assert code(batch(desc=None)) == A.AES_E_NULL
    assert code(batch(workspace=None)) == A.AES_E_NULL
    assert code(batch(nmsg=5)) == A.AES_E_ARG
    assert code(batch(max_msgs=0, nmsg=0)) == A.AES_E_ARG
    assert code(batch(nkeys=0)) == A.AES_E_ARG
    assert code(batch(in_base=0x300008)) == A.AES_E_ALIGN
    assert code(batch(workspace=0x500010)) == A.AES_E_ALIGN
    assert code(batch(workspace_bytes=ws - 1)) == A.AES_E_LENGTH
    assert code(batch(tile_blocks=-1)) == A.AES_E_ARG
    assert code(batch(tile_blocks=1025)) == A.AES_E_ARG
    assert code(batch(gcm=0x600004)) == A.AES_E_ALIGN
    for bpt in (1, 3, 8, -2):
        assert code(batch(blocks_per_thread=bpt)) == A.AES_E_ARG


def test_gcm_batch_layout(A):
    import ctypes
    assert A.GCM_DESC_DTYPE.itemsize == 32
    # the gcm pointer follows tile_blocks at the end of aes_batch
    assert A.aes_batch.gcm.offset == A.aes_batch.tile_blocks.offset + 4 == 96
    assert A.aes_batch.blocks_per_thread.offset == 104 and ctypes.sizeof(A.aes_batch) == 112
    assert A.AES_MODE_GCM == 4 and A.MODES["gcm"] == 4
    text = open(HEADER).read()
    assert "AES_MODE_GCM = 4" in text


def test_noalloc_batch_argument_checks(A):
    ws = A.aes_batch_workspace_size(4)
    f = dict(desc=0x100000, nmsg=4, d_nmsg=None, keys=0x200000, nkeys=4, in_base=0x300000, in_bytes=4096,
             out_base=0x400000, out_bytes=4096, workspace=None, workspace_bytes=0, max_msgs=4, tile_blocks=0)

    def code(**kw):
        with pytest.raises(A.AESError) as e:
            A.aes_batch_run_noalloc(A.aes_batch(**dict(f, **kw)), stream=0)
        return e.value.code

    assert code(workspace=0x500000, workspace_bytes=ws) == A.AES_E_ARG     # the library's workspace only
    assert code(workspace_bytes=ws) == A.AES_E_ARG
    assert code(max_msgs=A.AES_BATCH_NOALLOC_MAX_MSGS + 1) == A.AES_E_LENGTH
    assert A.lib.aes_batch_run_noalloc(None, None) == A.AES_E_NULL
    text = open(HEADER).read()
    assert "#define AES_BATCH_NOALLOC_MAX_MSGS %d" % A.AES_BATCH_NOALLOC_MAX_MSGS in text


def test_descriptor_layout(A):
    d = A.make_descs([16, 17, 0, 100], keybits=[128, 192, 256, 128], mode=["ecb", "ctr", "ctr", "ecb"],
                     decrypt=[0, 1, 0, 1])
    assert d.dtype.itemsize == 48
    assert list(d["in_off"]) == [0, 16, 48, 48]
    assert list(d["keybits_code"]) == [0, 1, 2, 0]
    assert list(d["mode"]) == [0, 1, 1, 0]
    raw = d.view(np.uint8).reshape(4, 48)
    assert raw[1, 8:16].view("<u8")[0] == 16       # out_off follows in_off
    assert raw[1, 28] == 1                          # keybits_code at byte 28


class _Refused:
    """Stands in for a library function that the binding must not reach."""

    def __call__(self, *args):
        raise AssertionError("the library was called")


@pytest.mark.parametrize("fn", ["aes_encrypt", "aes_decrypt", "aes_copy"])
def test_binding_checks_tensor_extents_before_the_library(A, monkeypatch, fn):
    # CPU tensors stand in for device tensors: every check here fails before
    # the binding would call into the library (which is replaced by a trap)
    import torch
    monkeypatch.setattr(A.lib, fn, _Refused())
    rk, nr = A.aes_expand_key(np.zeros(16, np.uint8))
    x, y = torch.zeros(64, dtype=torch.uint8), torch.zeros(64, dtype=torch.uint8)
    call = getattr(A, fn)
    args = (lambda i, o, n: (i, o, n)) if fn == "aes_copy" else (lambda i, o, n: (i, o, n, rk, nr, "ecb"))
    with pytest.raises(ValueError, match="holds 64 bytes"):
        call(*args(x, y, 80), stream=0)                           # beyond both tensors
    with pytest.raises(ValueError, match="out holds 48"):
        call(*args(x, y[:48], 64), stream=0)                      # beyond the output
    with pytest.raises(ValueError, match="contiguous"):
        call(*args(x.view(8, 8).t(), y, 64), stream=0)            # a strided view
    with pytest.raises(ValueError, match="device"):
        call(*args(x, y, 64), stream=0)                           # fits, but on the host
    with pytest.raises(ValueError, match=">= 0"):
        call(*args(x, y, -16), stream=0)


def test_binding_checks_xts_and_gcm_extents(A, monkeypatch):
    import torch
    for name in ("aes_xts_encrypt", "aes_gcm_encrypt", "aes_gcm_decrypt"):
        monkeypatch.setattr(A.lib, name, _Refused())
    rk, nr = A.aes_expand_key(np.zeros(16, np.uint8))
    x, y = torch.zeros(512, dtype=torch.uint8), torch.zeros(512, dtype=torch.uint8)
    with pytest.raises(ValueError, match="inp holds 512"):
        A.aes_xts_encrypt(x, y, 1024, rk, rk, nr, 512, stream=0)
    ws = torch.zeros(A.aes_gcm_workspace_size(), dtype=torch.uint8)
    tag, aad, ok = torch.zeros(16, dtype=torch.uint8), torch.zeros(32, dtype=torch.uint8), torch.zeros(1, dtype=torch.int32)
    with pytest.raises(ValueError, match="aad holds 32"):
        A.aes_gcm_encrypt(x, y, 512, aad, 48, rk, nr, bytes(12), tag, ws, stream=0)
    with pytest.raises(ValueError, match="tag holds 8"):
        A.aes_gcm_encrypt(x, y, 512, aad, 32, rk, nr, bytes(12), tag[:8], ws, stream=0)
    with pytest.raises(ValueError, match="workspace holds"):
        A.aes_gcm_encrypt(x, y, 512, aad, 32, rk, nr, bytes(12), tag, ws[:100], workspace_bytes=8192, stream=0)
    with pytest.raises(ValueError, match="ok holds 2"):
        A.aes_gcm_decrypt(x, y, 512, aad, 32, rk, nr, bytes(12), tag, 16, ok.view(torch.uint8)[:2], ws,
                          stream=0)
    with pytest.raises(ValueError, match="device"):
        A.aes_gcm_decrypt(x, y, 512, aad, 32, rk, nr, bytes(12), tag, 16, ok, ws, stream=0)


def test_batch_binding_picks_gcm_passes(A):
    # the binding asks for the one-pass GCM kernels only when a GCM message
    # has at least 2 x 65,536 GHASH blocks (additional data, ciphertext and
    # the length block)
    d = A.make_descs([16 * 131071, 16 * 131070, 5], mode="gcm", keybits=128)
    assert A._has_long_gcm(d, None)
    assert not A._has_long_gcm(d[1:], None)
    g = np.zeros(2, A.GCM_DESC_DTYPE)
    g["aad_bytes"] = [16, 0]
    assert A._has_long_gcm(d[1:], g)
    assert not A._has_long_gcm(A.make_descs([16 << 20], mode="ctr"), None)
