"""Python binding of libaesgpu (include/aesgpu.h): the same calls, with the
same names, marshalled through ctypes.

Only argument marshalling happens here: device buffers are torch tensors
(torch supplies device memory and streams), host arguments are numpy arrays
or bytes, and every step of the cipher runs in the library's HIP kernels.
There is no fallback: if the library is missing or fails to load, importing
this module raises.
"""
import ctypes
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

AES_MODE_ECB = 0
AES_MODE_CTR = 1

MODES = {"ecb": AES_MODE_ECB, "ctr": AES_MODE_CTR, AES_MODE_ECB: AES_MODE_ECB,
         AES_MODE_CTR: AES_MODE_CTR}

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
    "aes_last_error": (ctypes.c_char_p, []),
    "aes_set_launch": (ctypes.c_int, [ctypes.c_void_p]),
    "aes_get_launch": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p]),
    "aes_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_void_p]),
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
    _check(fn(_dptr(inp), _dptr(out), nbytes, _hptr(rk), Nr, mode, _hptr(c0),
              _stream_handle(stream, inp)))
    return out


def aes_encrypt(inp, out, nbytes, roundkeys, Nr, mode, ctr0=None, stream=None):
    """Enqueue encryption of nbytes of device buffer `inp` into `out`."""
    return _crypt(lib.aes_encrypt, inp, out, nbytes, roundkeys, Nr, mode, ctr0, stream)


def aes_decrypt(inp, out, nbytes, roundkeys, Nr, mode, ctr0=None, stream=None):
    """Enqueue decryption of nbytes of device buffer `inp` into `out`."""
    return _crypt(lib.aes_decrypt, inp, out, nbytes, roundkeys, Nr, mode, ctr0, stream)


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


def aes_get_launch(nbytes, mode=AES_MODE_ECB, decrypt=False):
    c = aes_launch()
    _check(lib.aes_get_launch(nbytes, _mode(mode), int(bool(decrypt)), ctypes.byref(c)))
    return c.as_dict()


def aes_copy(inp, out, nbytes=None, stream=None):
    if nbytes is None:
        nbytes = inp.numel() * inp.element_size()
    _check(lib.aes_copy(_dptr(inp), _dptr(out), nbytes, _stream_handle(stream, inp)))
    return out


# --- conveniences on top of the calls above (allocation through torch) ----
def encrypt(x, roundkeys, Nr, mode="ecb", ctr0=None, out=None, stream=None):
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_encrypt(x, out, x.numel() * x.element_size(), roundkeys, Nr, mode, ctr0, stream)


def decrypt(x, roundkeys, Nr, mode="ecb", ctr0=None, out=None, stream=None):
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_decrypt(x, out, x.numel() * x.element_size(), roundkeys, Nr, mode, ctr0, stream)
