"""An independent AES-XTS and AES-GCM for the oracle's pins: the system's
libcrypto (OpenSSL 3) called through its public EVP interface with ctypes.

The library is only called, never read: keys, IVs and data go in, the
ciphertext and tag come out.  CPU only; the tests that use it skip when the
library or one of its ciphers is missing.

XTS (IEEE 1619): the EVP key is K1 || K2 (data key, tweak key) and the EVP
IV is the 16-byte tweak block of one data unit; one EVP update enciphers one
data unit.  GCM (SP 800-38D): any IV length (set before the key), the
additional data as an update with no output, the tag read after the final
call (encryption) or set before it (decryption, which fails on a mismatch).
"""
import ctypes
import ctypes.util

import numpy as np

_EVP_CTRL_GCM_SET_IVLEN = 0x9
_EVP_CTRL_GCM_GET_TAG = 0x10
_EVP_CTRL_GCM_SET_TAG = 0x11

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib or None
    try:
        lib = ctypes.CDLL(ctypes.util.find_library("crypto") or "libcrypto.so.3")
        lib.EVP_CIPHER_fetch.restype = ctypes.c_void_p
        lib.EVP_CIPHER_fetch.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_char_p]
        lib.EVP_CIPHER_free.argtypes = [ctypes.c_void_p]
        lib.EVP_CIPHER_CTX_new.restype = ctypes.c_void_p
        lib.EVP_CIPHER_CTX_free.argtypes = [ctypes.c_void_p]
        lib.EVP_CipherInit_ex.restype = ctypes.c_int
        lib.EVP_CipherInit_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int]
        lib.EVP_CipherUpdate.restype = ctypes.c_int
        lib.EVP_CipherUpdate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                         ctypes.c_char_p, ctypes.c_int]
        lib.EVP_CipherFinal_ex.restype = ctypes.c_int
        lib.EVP_CipherFinal_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
        lib.EVP_CIPHER_CTX_ctrl.restype = ctypes.c_int
        lib.EVP_CIPHER_CTX_ctrl.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.EVP_CIPHER_CTX_set_padding.restype = ctypes.c_int
        lib.EVP_CIPHER_CTX_set_padding.argtypes = [ctypes.c_void_p, ctypes.c_int]
    except (OSError, AttributeError):
        _lib = False
        return None
    _lib = lib
    return lib


def available(name):
    """True if libcrypto loads and offers the cipher `name` (e.g. b"AES-128-XTS")."""
    lib = _load()
    if lib is None:
        return False
    c = lib.EVP_CIPHER_fetch(None, name, None)
    if not c:
        return False
    lib.EVP_CIPHER_free(c)
    return True


class _Ctx:
    def __init__(self, name):
        self.lib = _load()
        if self.lib is None:
            raise RuntimeError("libcrypto not available")
        self.cipher = self.lib.EVP_CIPHER_fetch(None, name, None)
        if not self.cipher:
            raise RuntimeError("libcrypto has no %r" % name)
        self.ctx = self.lib.EVP_CIPHER_CTX_new()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.lib.EVP_CIPHER_CTX_free(self.ctx)
        self.lib.EVP_CIPHER_free(self.cipher)

    def init(self, key, iv, enc, cipher=True):
        ok = self.lib.EVP_CipherInit_ex(self.ctx, self.cipher if cipher else None, None,
                                        None if key is None else bytes(key), None if iv is None else bytes(iv),
                                        int(enc))
        if ok != 1:
            raise RuntimeError("EVP_CipherInit_ex failed")

    def update(self, data, want_out=True):
        data = bytes(data)
        out = ctypes.create_string_buffer(len(data) + 32) if want_out else None
        n = ctypes.c_int(0)
        if self.lib.EVP_CipherUpdate(self.ctx, out, ctypes.byref(n), data, len(data)) != 1:
            raise RuntimeError("EVP_CipherUpdate failed")
        return out.raw[:n.value] if want_out else b""

    def final(self):
        out = ctypes.create_string_buffer(32)
        n = ctypes.c_int(0)
        ok = self.lib.EVP_CipherFinal_ex(self.ctx, out, ctypes.byref(n))
        return ok == 1, out.raw[:n.value]

    def ctrl(self, op, arg, ptr):
        return self.lib.EVP_CIPHER_CTX_ctrl(self.ctx, op, arg, ptr)


def xts_unit(key1, key2, tweak16, data, decrypt=False):
    """One data unit (whole blocks, at least one) through libcrypto's XTS:
    key1 the data key, key2 the tweak key (same size, 16 or 32 bytes),
    tweak16 the 16-byte tweak block."""
    k1, k2 = bytes(key1), bytes(key2)
    name = b"AES-128-XTS" if len(k1) == 16 else b"AES-256-XTS"
    with _Ctx(name) as c:
        c.init(k1 + k2, bytes(tweak16), not decrypt)
        out = c.update(data)
        ok, rest = c.final()
        if not ok:
            raise RuntimeError("XTS final failed")
    return np.frombuffer(out + rest, np.uint8).copy()


def gcm_encrypt(key, iv, aad, data):
    """Returns (ciphertext, 16-byte tag)."""
    k = bytes(key)
    with _Ctx({16: b"AES-128-GCM", 24: b"AES-192-GCM", 32: b"AES-256-GCM"}[len(k)]) as c:
        c.init(None, None, True)
        if c.ctrl(_EVP_CTRL_GCM_SET_IVLEN, len(bytes(iv)), None) != 1:
            raise RuntimeError("IV length rejected")
        c.init(k, iv, True, cipher=False)
        if len(bytes(aad)):
            c.update(aad, want_out=False)
        out = c.update(data) if len(bytes(data)) else b""
        ok, rest = c.final()
        tag = ctypes.create_string_buffer(16)
        if not ok or c.ctrl(_EVP_CTRL_GCM_GET_TAG, 16, tag) != 1:
            raise RuntimeError("GCM final failed")
    return np.frombuffer(out + rest, np.uint8).copy(), np.frombuffer(tag.raw, np.uint8).copy()


def gcm_decrypt(key, iv, aad, data, tag):
    """Returns (plaintext, authentic?) for a tag of len(tag) bytes."""
    k, t = bytes(key), bytes(tag)
    with _Ctx({16: b"AES-128-GCM", 24: b"AES-192-GCM", 32: b"AES-256-GCM"}[len(k)]) as c:
        c.init(None, None, False)
        if c.ctrl(_EVP_CTRL_GCM_SET_IVLEN, len(bytes(iv)), None) != 1:
            raise RuntimeError("IV length rejected")
        c.init(k, iv, False, cipher=False)
        if len(bytes(aad)):
            c.update(aad, want_out=False)
        out = c.update(data) if len(bytes(data)) else b""
        tb = ctypes.create_string_buffer(t, len(t))
        if c.ctrl(_EVP_CTRL_GCM_SET_TAG, len(t), tb) != 1:
            raise RuntimeError("tag length rejected")
        ok, rest = c.final()
    return np.frombuffer(out + rest, np.uint8).copy(), ok
