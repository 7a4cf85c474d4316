"""Python binding of libaesgpu (include/aesgpu.h): the same calls, with the
same names, marshalled through ctypes.

Only argument marshalling happens here: device buffers are torch tensors
(torch supplies device memory and streams), host arguments are numpy arrays
or bytes, and every step of the cipher runs in the library's HIP kernels.
There is no fallback: if the library is missing or fails to load, importing
this module raises.
"""
import ctypes
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaesgpu.so")

AES_OK = 0
AES_E_NULL = 1
AES_E_KEYBITS = 2
AES_E_NR = 3
AES_E_LENGTH = 4
AES_E_ALIGN = 5
AES_E_OVERLAP = 6
AES_E_MODE = 7
AES_E_DEVICE = 8
AES_E_ARG = 9
AES_E_BUDGET = 10

AES_MODE_ECB = 0
AES_MODE_CTR = 1
AES_MODE_CBC = 2
AES_MODE_XTS = 3      # batch descriptors only
AES_MODE_GCM = 4      # batch descriptors and served requests only

MODES = {"ecb": AES_MODE_ECB, "ctr": AES_MODE_CTR, "cbc": AES_MODE_CBC, "xts": AES_MODE_XTS,
         "gcm": AES_MODE_GCM}

# every function the header declares, with its ctypes signature
_SIGNATURES = {
    "aes_expand_key": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_int)]),
    "aes_encrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "aes_decrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "aes_xts_encrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_size_t, ctypes.c_uint64, ctypes.c_void_p]),
    "aes_xts_decrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_size_t, ctypes.c_uint64, ctypes.c_void_p]),
    "aes_gcm_workspace_size": (ctypes.c_int, [ctypes.POINTER(ctypes.c_size_t)]),
    "aes_gcm_encrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "aes_gcm_decrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "aes_last_error": (ctypes.c_char_p, []),
    "aes_set_launch": (ctypes.c_int, [ctypes.c_void_p]),
    "aes_get_launch": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p]),
    "aes_set_tuned": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "aes_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_void_p]),
    "aes_lds_gather": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.c_void_p]),
    "aes_lds_gather_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                             ctypes.c_void_p]),
    "aes_batch_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "aes_batch_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "aes_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "aes_batch_run_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "aes_batch_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64)]),
    "aes_batch_graph_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "aes_batch_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "aes_batch_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "aes_serve_scratch_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "aes_serve_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
}


class AESError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("aesgpu error %d: %s" % (code, message))
        self.code = code


class aes_launch(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int), ("blocks_per_thread", ctypes.c_int),
                ("wg_size", ctypes.c_int), ("grid", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# aes_msg_desc, as a numpy record so that whole descriptor tables are built
# with array operations
MSG_DESC_DTYPE = np.dtype([("in_off", "<u8"), ("out_off", "<u8"), ("nbytes", "<u8"),
                           ("key_idx", "<u4"), ("keybits_code", "u1"), ("mode", "u1"),
                           ("decrypt", "u1"), ("reserved", "u1"), ("ctr0", "u1", (16,))])
assert MSG_DESC_DTYPE.itemsize == 48


# aes_gcm_desc: the GCM fields of a batch message
GCM_DESC_DTYPE = np.dtype([("aad_off", "<u8"), ("aad_bytes", "<u8"), ("tag_off", "<u8"),
                           ("tag_bytes", "<u4"), ("ok", "<i4")])
assert GCM_DESC_DTYPE.itemsize == 32


class aes_batch(ctypes.Structure):
    _fields_ = [("desc", ctypes.c_void_p), ("nmsg", ctypes.c_int), ("d_nmsg", ctypes.c_void_p),
                ("keys", ctypes.c_void_p), ("nkeys", ctypes.c_int),
                ("in_base", ctypes.c_void_p), ("in_bytes", ctypes.c_uint64),
                ("out_base", ctypes.c_void_p), ("out_bytes", ctypes.c_uint64),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("max_msgs", ctypes.c_int), ("tile_blocks", ctypes.c_int), ("gcm", ctypes.c_void_p),
                ("blocks_per_thread", ctypes.c_int), ("gcm_two_pass", ctypes.c_int)]


# aes_request and aes_request_result, as numpy records
REQUEST_DTYPE = np.dtype([("arrival_s", "<f8"), ("nbytes", "<u8"), ("payload_seed", "<u8"),
                          ("key_idx", "<u4"), ("keybits_code", "u1"), ("mode", "u1"),
                          ("decrypt", "u1"), ("reserved", "u1"), ("ctr0", "u1", (16,))])
RESULT_DTYPE = np.dtype([("latency_s", "<f8"), ("admit_s", "<f8"), ("in_off", "<u8"),
                         ("out_off", "<u8"), ("status", "<i4"), ("launch", "<i4"),
                         ("overwritten", "<i4"), ("authentic", "<i4")])
assert REQUEST_DTYPE.itemsize == 48 and RESULT_DTYPE.itemsize == 48


class aes_serve_cfg(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int), ("budget_bytes", ctypes.c_uint64),
                ("max_batch_msgs", ctypes.c_int), ("tile_blocks", ctypes.c_int),
                ("blocks_per_thread", ctypes.c_int),
                ("timeout_s", ctypes.c_double), ("simulate_gbps", ctypes.c_double)]


class aes_serve_stats(ctypes.Structure):
    _fields_ = [("span_s", ctypes.c_double), ("bytes_done", ctypes.c_uint64),
                ("completed", ctypes.c_int), ("rejected", ctypes.c_int),
                ("launches", ctypes.c_int), ("max_inflight_reqs", ctypes.c_int),
                ("max_inflight_bytes", ctypes.c_uint64), ("fill_device_s", ctypes.c_double),
                ("cipher_device_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libaesgpu.so is not built (expected at %s); run "
                          "`python -m paper_1403_7295_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()
TUNED_TABLE = os.path.join(HERE, "tuned_gfx950.json")
TUNED_TILE_BLOCKS = 0      # batch split step picked by the autotuner (0 = library default)
TUNED_BATCH_BPT = 0        # batch blocks per thread picked by the autotuner (0 = library default)


def _check(status):
    if status != AES_OK:
        raise AESError(status, lib.aes_last_error().decode(errors="replace"))


def _host_bytes(a, n=None):
    """Host argument as a ctypes-addressable uint8 numpy array."""
    if a is None:
        return None
    if isinstance(a, (bytes, bytearray, memoryview)):
        arr = np.frombuffer(bytes(a), dtype=np.uint8).copy()
    else:
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.uint8)).reshape(-1)
    if n is not None and arr.size < n:
        raise ValueError("host argument needs %d bytes, got %d" % (n, arr.size))
    return arr


def _hptr(arr):
    return None if arr is None else arr.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    """Device address of a torch tensor, or an int taken as an address."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _nbytes_arg(n, name="nbytes"):
    n = int(n)
    if n < 0:
        raise ValueError("%s must be >= 0, got %d" % (name, n))
    return n


def _dev(*specs):
    """Device addresses of buffer arguments, each given as (tensor, bytes the
    call will touch, name).  Checked here before any library call, since the
    kernels trust the extents they are given: every torch tensor must hold
    its bytes (all extents are checked first), be contiguous, and live on
    the device (CUDA).  An int is taken as a raw device address, which the
    caller vouches for; None stays None (a NULL pointer, which the library
    refuses where it needs one).  One address for one spec, else a list."""
    tensors = [(t, need, name) for t, need, name in specs if t is not None and not isinstance(t, int)]
    for t, need, name in tensors:
        have = t.numel() * t.element_size()
        if need > have:
            raise ValueError("%s holds %d bytes but the call would touch %d" % (name, have, need))
    for t, _, name in tensors:
        if not t.is_contiguous():
            raise ValueError("%s must be a contiguous tensor" % name)
    for t, _, name in tensors:
        if not t.is_cuda:
            raise ValueError("%s must be a device (CUDA) tensor, not %s" % (name, t.device))
    ptrs = [t if t is None or isinstance(t, int) else t.data_ptr() for t, _, _ in specs]
    return ptrs[0] if len(ptrs) == 1 else ptrs


def _stream_handle(stream, like=None):
    if stream is None:
        import torch
        dev = like.device if like is not None and hasattr(like, "device") else None
        return torch.cuda.current_stream(dev).cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def aes_expand_key(key, keybits=None):
    """Key Expansion on the host.  Returns (round key bytes as numpy uint8, Nr)."""
    k = _host_bytes(key)
    keybits = keybits or 8 * k.size
    if k.size * 8 < keybits:
        raise ValueError("key shorter than keybits")
    rk = np.zeros(240, np.uint8)
    nr = ctypes.c_int(0)
    _check(lib.aes_expand_key(_hptr(k), keybits, _hptr(rk), ctypes.byref(nr)))
    return rk[:16 * (nr.value + 1)].copy(), nr.value


def _mode(mode):
    # names map to their codes; integers go through unchanged for the library to check
    return mode if isinstance(mode, int) else MODES[mode]


def _crypt(fn, inp, out, nbytes, roundkeys, Nr, mode, ctr0, stream):
    mode = _mode(mode)
    rk = _host_bytes(roundkeys)
    c0 = _host_bytes(ctr0, 16) if ctr0 is not None else None
    if nbytes is None:
        nbytes = inp.numel() * inp.element_size()
    nbytes = _nbytes_arg(nbytes)
    pi, po = _dev((inp, nbytes, "inp"), (out, nbytes, "out"))
    _check(fn(pi, po, nbytes, _hptr(rk), Nr, mode, _hptr(c0), _stream_handle(stream, inp)))
    return out


def aes_encrypt(inp, out, nbytes, roundkeys, Nr, mode, ctr0=None, stream=None):
    """Enqueue encryption of nbytes of device buffer `inp` into `out`."""
    return _crypt(lib.aes_encrypt, inp, out, nbytes, roundkeys, Nr, mode, ctr0, stream)


def aes_decrypt(inp, out, nbytes, roundkeys, Nr, mode, ctr0=None, stream=None):
    """Enqueue decryption of nbytes of device buffer `inp` into `out`."""
    return _crypt(lib.aes_decrypt, inp, out, nbytes, roundkeys, Nr, mode, ctr0, stream)


def _xts(fn, inp, out, nbytes, roundkeys1, roundkeys2, Nr, unit_bytes, first_unit, stream):
    rk1, rk2 = _host_bytes(roundkeys1), _host_bytes(roundkeys2)
    if nbytes is None:
        nbytes = inp.numel() * inp.element_size()
    nbytes = _nbytes_arg(nbytes)
    pi, po = _dev((inp, nbytes, "inp"), (out, nbytes, "out"))
    _check(fn(pi, po, nbytes, _hptr(rk1), _hptr(rk2), Nr, unit_bytes, first_unit,
              _stream_handle(stream, inp)))
    return out


def aes_xts_encrypt(inp, out, nbytes, roundkeys1, roundkeys2, Nr, unit_bytes, first_unit=0, stream=None):
    """Enqueue XTS encryption of nbytes (data units of unit_bytes; tweak
    values first_unit, first_unit + 1, ...)."""
    return _xts(lib.aes_xts_encrypt, inp, out, nbytes, roundkeys1, roundkeys2, Nr, unit_bytes,
                first_unit, stream)


def aes_xts_decrypt(inp, out, nbytes, roundkeys1, roundkeys2, Nr, unit_bytes, first_unit=0, stream=None):
    """Enqueue XTS decryption; the arguments of aes_xts_encrypt."""
    return _xts(lib.aes_xts_decrypt, inp, out, nbytes, roundkeys1, roundkeys2, Nr, unit_bytes,
                first_unit, stream)


def aes_gcm_workspace_size():
    n = ctypes.c_size_t(0)
    _check(lib.aes_gcm_workspace_size(ctypes.byref(n)))
    return n.value


def aes_gcm_encrypt(inp, out, nbytes, aad, aad_bytes, roundkeys, Nr, iv, tag, workspace,
                    workspace_bytes=None, stream=None):
    """Enqueue GCM encryption; the 16-byte tag goes to device buffer `tag`."""
    rk, v = _host_bytes(roundkeys), _host_bytes(iv)
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    nbytes, aad_bytes = _nbytes_arg(nbytes), _nbytes_arg(aad_bytes, "aad_bytes")
    workspace_bytes = _nbytes_arg(workspace_bytes, "workspace_bytes")
    pi, po, pa, pt, pw = _dev((inp, nbytes, "inp"), (out, nbytes, "out"), (aad, aad_bytes, "aad"),
                              (tag, 16, "tag"), (workspace, workspace_bytes, "workspace"))
    args = (pi, po, nbytes, pa, aad_bytes, _hptr(rk), Nr, _hptr(v), v.size, pt, pw, workspace_bytes)
    _check(lib.aes_gcm_encrypt(*args, _stream_handle(stream, tag)))
    return out


def aes_gcm_decrypt(inp, out, nbytes, aad, aad_bytes, roundkeys, Nr, iv, tag, tag_bytes, ok, workspace,
                    workspace_bytes=None, stream=None):
    """Enqueue GCM decryption; device int32 `ok` receives 1 if the tag matches."""
    rk, v = _host_bytes(roundkeys), _host_bytes(iv)
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    nbytes, aad_bytes = _nbytes_arg(nbytes), _nbytes_arg(aad_bytes, "aad_bytes")
    workspace_bytes = _nbytes_arg(workspace_bytes, "workspace_bytes")
    tag_bytes = _nbytes_arg(tag_bytes, "tag_bytes")
    pi, po, pa, pt, pk, pw = _dev((inp, nbytes, "inp"), (out, nbytes, "out"), (aad, aad_bytes, "aad"),
                                  (tag, tag_bytes, "tag"), (ok, 4, "ok"),
                                  (workspace, workspace_bytes, "workspace"))
    args = (pi, po, nbytes, pa, aad_bytes, _hptr(rk), Nr, _hptr(v), v.size, pt, tag_bytes, pk, pw,
            workspace_bytes)
    _check(lib.aes_gcm_decrypt(*args, _stream_handle(stream, tag)))
    return out


def aes_last_error():
    return lib.aes_last_error().decode(errors="replace")


def aes_set_launch(cfg=None, **fields):
    """Force a launch configuration (dict or keyword fields); None clears it."""
    if cfg is None and not fields:
        _check(lib.aes_set_launch(None))
        return
    c = aes_launch()
    for k, v in dict(cfg or {}, **fields).items():
        setattr(c, k, int(v))
    _check(lib.aes_set_launch(ctypes.byref(c)))


def aes_get_launch(nbytes, mode=AES_MODE_ECB, decrypt=False, Nr=10):
    c = aes_launch()
    _check(lib.aes_get_launch(nbytes, _mode(mode), int(bool(decrypt)), Nr, ctypes.byref(c)))
    return c.as_dict()


class aes_tuned_entry(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("decrypt", ctypes.c_int), ("Nr", ctypes.c_int),
                ("min_bytes", ctypes.c_uint64), ("cfg", aes_launch)]


def aes_set_tuned(entries):
    """Install a tuned table: entries are dicts with mode, decrypt, Nr,
    min_bytes and cfg (an aes_launch dict)."""
    arr = (aes_tuned_entry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i].mode = _mode(e["mode"])
        arr[i].decrypt = int(e["decrypt"])
        arr[i].Nr = int(e["Nr"])
        arr[i].min_bytes = int(e["min_bytes"])
        for k, v in e["cfg"].items():
            setattr(arr[i].cfg, k, int(v))
    _check(lib.aes_set_tuned(arr, len(entries)))


def aes_copy(inp, out, nbytes=None, stream=None):
    if nbytes is None:
        nbytes = inp.numel() * inp.element_size()
    nbytes = _nbytes_arg(nbytes)
    pi, po = _dev((inp, nbytes, "inp"), (out, nbytes, "out"))
    _check(lib.aes_copy(pi, po, nbytes, _stream_handle(stream, inp)))
    return out


LDS_GATHER_RECORD_BYTES = 24   # aes_lds_gather_stat: cycles, ticks (uint64), fold, pad (uint32)


def aes_lds_gather(out, rounds, stream=None, layout=0):
    """Runs the LDS gather calibration kernel over table layout 0 (four
    tables x 32 copies) or 3 (one table x 64 copies, two workgroups per
    compute unit); `out` is a device tensor holding one 24-byte record per
    wave.  Returns (waves, constant-rate clock in kHz)."""
    waves, khz = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib.aes_lds_gather_layout(_dev((out, 0, "out")), out.numel() * out.element_size(), int(rounds),
                                     int(layout), ctypes.byref(waves), ctypes.byref(khz),
                                     _stream_handle(stream, out)))
    return waves.value, khz.value


# --- conveniences on top of the calls above (allocation through torch) ----
def encrypt(x, roundkeys, Nr, mode="ecb", ctr0=None, out=None, stream=None):
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_encrypt(x, out, x.numel() * x.element_size(), roundkeys, Nr, mode, ctr0, stream)


def decrypt(x, roundkeys, Nr, mode="ecb", ctr0=None, out=None, stream=None):
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_decrypt(x, out, x.numel() * x.element_size(), roundkeys, Nr, mode, ctr0, stream)


# --- batches ----------------------------------------------------------------
def aes_batch_workspace_size(max_msgs):
    n = ctypes.c_size_t(0)
    _check(lib.aes_batch_workspace_size(max_msgs, ctypes.byref(n)))
    return n.value


def aes_batch_plan(nmsg, d_desc=None):
    """Workspace bytes of a batch of nmsg messages (the descriptor table is
    not read: the size depends on the count only)."""
    n = ctypes.c_size_t(0)
    _check(lib.aes_batch_plan(_dptr(d_desc), int(nmsg), ctypes.byref(n)))
    return n.value


def aes_batch_run(batch, stream=None):
    _check(lib.aes_batch_run(ctypes.byref(batch), _stream_handle(stream)))


AES_BATCH_NOALLOC_MAX_MSGS = 16384


def aes_batch_run_noalloc(batch, stream=None):
    """aes_batch_run with the library's own workspace (batch.workspace must
    be None and workspace_bytes 0); allocates nothing."""
    _check(lib.aes_batch_run_noalloc(ctypes.byref(batch), _stream_handle(stream)))


def aes_batch_query(batch, stream=None):
    """Waits for `stream`; returns (messages planned, messages rejected)."""
    t, r = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib.aes_batch_query(ctypes.byref(batch), _stream_handle(stream), ctypes.byref(t),
                               ctypes.byref(r)))
    return t.value, r.value


def aes_batch_graph_create(batch):
    g = ctypes.c_void_p(0)
    _check(lib.aes_batch_graph_create(ctypes.byref(batch), ctypes.byref(g)))
    return g


def aes_batch_graph_launch(graph, stream=None):
    _check(lib.aes_batch_graph_launch(graph, _stream_handle(stream)))


def aes_batch_graph_destroy(graph):
    _check(lib.aes_batch_graph_destroy(graph))


def make_descs(nbytes, in_off=None, out_off=None, key_idx=None, keybits=128, mode="ecb",
               decrypt=False, ctr0=None):
    """Descriptor table (numpy, MSG_DESC_DTYPE) for messages of the given
    lengths.  Offsets default to the messages packed back to back, each
    starting on a 16-byte boundary; scalars broadcast over messages."""
    nbytes = np.asarray(nbytes, dtype=np.uint64).reshape(-1)
    n = nbytes.size
    d = np.zeros(n, MSG_DESC_DTYPE)
    d["nbytes"] = nbytes
    if in_off is None:
        padded = (nbytes + np.uint64(15)) // np.uint64(16) * np.uint64(16)
        in_off = np.concatenate([[0], np.cumsum(padded)[:-1]]).astype(np.uint64) if n else padded
    d["in_off"] = in_off
    d["out_off"] = in_off if out_off is None else out_off
    d["key_idx"] = np.arange(n) if key_idx is None else key_idx
    kb = np.broadcast_to(np.asarray(keybits), (n,))
    d["keybits_code"] = (kb.astype(np.int64) - 128) // 64
    md = np.broadcast_to(np.asarray(mode), (n,))
    d["mode"] = [_mode(m) for m in md] if md.dtype.kind in "UO" else md
    d["decrypt"] = np.broadcast_to(np.asarray(decrypt, dtype=np.uint8), (n,))
    if ctr0 is not None:
        d["ctr0"] = np.broadcast_to(np.asarray(ctr0, dtype=np.uint8), (n, 16))
    return d


def xts_ctr0(first_unit, key2_idx, unit_bytes):
    """The ctr0 field of an XTS batch descriptor: tweak value of the first data
    unit, key slot of the tweak key, data-unit size (little-endian)."""
    return np.frombuffer(int(first_unit).to_bytes(8, "little") + int(key2_idx).to_bytes(4, "little") +
                         int(unit_bytes).to_bytes(4, "little"), dtype=np.uint8).copy()


# GCM messages of at least this many GHASH blocks (additional data,
# ciphertext, the length block) can take the library's one-pass kernels
GCM_ONE_PASS_MIN_BLOCKS = 2 * 65536


def _has_long_gcm(descs, gcm):
    """Whether a GCM descriptor is long enough for the one-pass kernels
    (additional data counted when its fields are given)."""
    m = descs["mode"] == AES_MODE_GCM
    if not m.any():
        return False
    pos = (descs["nbytes"][m].astype(np.uint64) + 15) // 16 + 1
    if gcm is not None:
        pos = pos + (np.asarray(gcm["aad_bytes"])[m].astype(np.uint64) + 15) // 16
    return bool((pos >= GCM_ONE_PASS_MIN_BLOCKS).any())


class Batch:
    """A batch of messages on the device: descriptors, keys and workspace held
    in torch tensors (torch supplies the memory), run through
    aes_batch_run or a captured graph.

    descs      numpy MSG_DESC_DTYPE array (see make_descs)
    keys       numpy uint8 array (nkeys, 32): one key per 32-byte slot
    inp, out   device tensors the descriptors' offsets point into
    gcm        numpy GCM_DESC_DTYPE array, one entry per message (GCM
               messages' additional data and tags), or None
    """

    def __init__(self, descs, keys, inp, out, tile_blocks=0, max_msgs=None, device=None, gcm=None,
                 blocks_per_thread=0, gcm_two_pass=None):
        import torch
        self.device = device or inp.device
        _dev((inp, 0, "inp"), (out, 0, "out"))
        descs = np.ascontiguousarray(descs, dtype=MSG_DESC_DTYPE)
        keys = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 32)
        self.max_msgs = max(1, int(max_msgs or len(descs)))
        self.tile_blocks = int(tile_blocks or TUNED_TILE_BLOCKS)
        self.d_desc = torch.zeros(self.max_msgs * 48, dtype=torch.uint8, device=self.device)
        self.d_nmsg = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.d_keys = torch.from_numpy(keys.reshape(-1).copy()).to(self.device)
        ws = aes_batch_workspace_size(self.max_msgs)
        self.workspace = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.inp, self.out = inp, out
        self.c = aes_batch(desc=self.d_desc.data_ptr(), nmsg=0, d_nmsg=None,
                           keys=self.d_keys.data_ptr(), nkeys=keys.shape[0],
                           in_base=inp.data_ptr(), in_bytes=inp.numel() * inp.element_size(),
                           out_base=out.data_ptr(), out_bytes=out.numel() * out.element_size(),
                           workspace=aligned, workspace_bytes=ws, max_msgs=self.max_msgs,
                           tile_blocks=self.tile_blocks,
                           blocks_per_thread=int(blocks_per_thread or TUNED_BATCH_BPT))
        self.d_gcm = None
        if gcm is not None:
            self.d_gcm = torch.zeros(self.max_msgs * GCM_DESC_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
            self.c.gcm = self.d_gcm.data_ptr()
        # None: two passes for every GCM message unless the descriptors hold
        # one long enough for the one-pass kernels (a launch choice only)
        self.gcm_two_pass = gcm_two_pass
        self.graph = None
        self.set_descs(descs, gcm=gcm)

    def set_descs(self, descs, keys=None, stream=None, gcm=None):
        """Rewrite the descriptors (and optionally the keys and GCM fields) in place."""
        import torch
        descs = np.ascontiguousarray(descs, dtype=MSG_DESC_DTYPE)
        if len(descs) > self.max_msgs:
            raise ValueError("batch holds at most %d messages" % self.max_msgs)
        if gcm is not None:
            if self.d_gcm is None:
                raise ValueError("this batch was made without GCM fields")
            g = np.ascontiguousarray(gcm, dtype=GCM_DESC_DTYPE)
            if len(g) != len(descs):
                raise ValueError("one GCM entry per message")
            graw = torch.from_numpy(g.view(np.uint8).reshape(-1).copy())
            self.d_gcm[:graw.numel()].copy_(graw)
        raw = torch.from_numpy(descs.view(np.uint8).reshape(-1).copy())
        self.d_desc[:raw.numel()].copy_(raw)
        self.d_nmsg.fill_(len(descs))
        self.c.nmsg = len(descs)
        if self.gcm_two_pass is None:
            self.c.gcm_two_pass = 0 if _has_long_gcm(descs, gcm) else 1
        else:
            self.c.gcm_two_pass = int(bool(self.gcm_two_pass))
        if keys is not None:
            k = torch.from_numpy(np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1).copy())
            self.d_keys[:k.numel()].copy_(k)

    def run(self, stream=None):
        aes_batch_run(self.c, stream)

    def gcm_results(self, n):
        """The GCM fields of the first n messages as the device left them
        (after the stream has run the batch): ok holds each verdict."""
        return self.d_gcm[:n * GCM_DESC_DTYPE.itemsize].cpu().numpy().view(GCM_DESC_DTYPE).copy()

    def query(self, stream=None):
        return aes_batch_query(self.c, stream)

    def capture(self):
        """Capture the batch as a graph whose message count is read from the
        device at each launch."""
        if self.graph is None:
            c = aes_batch.from_buffer_copy(self.c)
            c.d_nmsg = self.d_nmsg.data_ptr()
            self.graph_c = c
            self.graph = aes_batch_graph_create(c)
        return self.graph

    def launch_graph(self, stream=None):
        aes_batch_graph_launch(self.capture(), stream)

    def close(self):
        if self.graph is not None:
            aes_batch_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- serving ----------------------------------------------------------------
def serve_cfg(streams=4, budget_bytes=8 << 30, max_batch_msgs=4096, tile_blocks=None,
              timeout_s=0.0, simulate_gbps=0.0, blocks_per_thread=None):
    """A request-loop configuration; tile_blocks and blocks_per_thread None
    take the autotuner's choices, the ones Batch uses too."""
    if tile_blocks is None:
        tile_blocks = TUNED_TILE_BLOCKS
    if blocks_per_thread is None:
        blocks_per_thread = TUNED_BATCH_BPT
    return aes_serve_cfg(streams=streams, budget_bytes=budget_bytes,
                         max_batch_msgs=max_batch_msgs, tile_blocks=tile_blocks,
                         blocks_per_thread=blocks_per_thread,
                         timeout_s=timeout_s, simulate_gbps=simulate_gbps)


def aes_serve_scratch_size(cfg):
    n = ctypes.c_size_t(0)
    _check(lib.aes_serve_scratch_size(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def aes_serve_run(reqs, cfg, d_keys=None, nkeys=None, scratch=None):
    """Run the request loop.  reqs: numpy REQUEST_DTYPE array sorted by
    arrival; d_keys: device tensor of 32-byte key slots; scratch: device
    tensor of at least aes_serve_scratch_size(cfg) bytes (256-byte aligned
    address).  Returns (results as RESULT_DTYPE array, stats dict)."""
    reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
    res = np.zeros(len(reqs), RESULT_DTYPE)
    st = aes_serve_stats()
    if nkeys is None:
        nkeys = (d_keys.numel() // 32) if d_keys is not None else 1 << 30
    sptr = _dptr(scratch)
    sbytes = 0 if scratch is None else scratch.numel() * scratch.element_size()
    _check(lib.aes_serve_run(reqs.ctypes.data_as(ctypes.c_void_p), len(reqs), _dptr(d_keys), nkeys,
                             sptr, sbytes, ctypes.byref(cfg), res.ctypes.data_as(ctypes.c_void_p),
                             ctypes.byref(st)))
    return res, st.as_dict()


class Server:
    """Device memory for the request loop (keys and scratch as torch tensors)
    and a run() that replays a request schedule through aes_serve_run."""

    def __init__(self, keys, cfg, device="cuda"):
        import torch
        self.cfg = cfg
        keys = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 32)
        self.nkeys = keys.shape[0]
        self.d_keys = torch.from_numpy(keys.reshape(-1).copy()).to(device)
        n = aes_serve_scratch_size(cfg)
        self._raw = torch.empty(n + 256, dtype=torch.uint8, device=device)
        off = (-self._raw.data_ptr()) % 256
        self.scratch = self._raw[off:off + n]

    def run(self, reqs):
        return aes_serve_run(reqs, self.cfg, self.d_keys, self.nkeys, self.scratch)

    def output(self, result, nbytes):
        """The output bytes of one finished request (a view into the arena)."""
        o = int(result["out_off"])
        return self.scratch[o:o + int(nbytes)]

    def tag(self, result, nbytes):
        """The tag an encrypting GCM request wrote after its output."""
        o = int(result["out_off"]) + (int(nbytes) + 15) // 16 * 16
        return self.scratch[o:o + 16]


def _install_tuned():
    """Install the autotuner's committed launch table for gfx950 (the only
    device the library runs on); host-side only, no device is touched."""
    global TUNED_TILE_BLOCKS, TUNED_BATCH_BPT
    if not os.path.exists(TUNED_TABLE):
        return
    with open(TUNED_TABLE) as f:
        table = json.load(f)
    aes_set_tuned([dict(mode=e["mode"], decrypt=e["decrypt"], Nr=e["Nr"], min_bytes=e["min_bytes"],
                        cfg=e["cfg"]) for e in table.get("entries", [])])
    TUNED_TILE_BLOCKS = int(table.get("batch_tile_blocks", 0))
    TUNED_BATCH_BPT = int(table.get("batch_blocks_per_thread", 0))


_install_tuned()
