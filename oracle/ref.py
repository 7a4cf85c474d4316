"""Python access to the oracle (a plain byte-oriented CPU AES, FIPS-197).

TEST INFRASTRUCTURE ONLY: the tests, the package's smoke check and the
benchmark's CPU-baseline leg are its only users.  It never imports the GPU
package and the GPU package never imports it.

Buffers are numpy ``uint8`` arrays (or ``bytes``); results come back as new
numpy arrays.  Every call goes straight to the C functions of ``aes_ref.c`` and
``par_run.c``; this file only marshals arguments.
"""
import ctypes
import os

import numpy as np

from . import build as _build

OP_ECB_ENC, OP_ECB_DEC, OP_CTR = 0, 1, 2

_u8p = ctypes.POINTER(ctypes.c_uint8)


def _ptr(a):
    return a.ctypes.data_as(_u8p)


def _as_u8(data):
    if isinstance(data, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(data), dtype=np.uint8)
    a = np.ascontiguousarray(data)
    if a.dtype != np.uint8:
        raise TypeError("oracle buffers are uint8")
    return a.reshape(-1)


class Oracle:
    """One loaded copy of the oracle library."""

    def __init__(self, path=None):
        path = path or _build.DEFAULT_LIB
        if not os.path.exists(path):
            _build.build(path)
        lib = ctypes.CDLL(path)
        lib.ref_xtime.restype = ctypes.c_uint8
        lib.ref_xtime.argtypes = [ctypes.c_uint8]
        lib.ref_gf_mul.restype = ctypes.c_uint8
        lib.ref_gf_mul.argtypes = [ctypes.c_uint8, ctypes.c_uint8]
        lib.ref_rcon.restype = ctypes.c_uint8
        lib.ref_rcon.argtypes = [ctypes.c_int]
        lib.ref_sbox.argtypes = [_u8p]
        lib.ref_inv_sbox.argtypes = [_u8p]
        for name in ("sub_bytes", "inv_sub_bytes", "shift_rows", "inv_shift_rows",
                     "mix_columns", "inv_mix_columns"):
            getattr(lib, "ref_step_" + name).argtypes = [_u8p]
        lib.ref_expand_key.restype = ctypes.c_int
        lib.ref_expand_key.argtypes = [_u8p, ctypes.c_int, _u8p]
        lib.ref_encrypt_block.argtypes = [_u8p, ctypes.c_int, _u8p, _u8p]
        lib.ref_decrypt_block.argtypes = [_u8p, ctypes.c_int, _u8p, _u8p]
        lib.ref_ecb.restype = ctypes.c_int
        lib.ref_ecb.argtypes = [ctypes.c_int, _u8p, ctypes.c_int, _u8p, _u8p, ctypes.c_size_t]
        lib.ref_ctr_block.argtypes = [_u8p, ctypes.c_uint64, _u8p]
        lib.ref_ctr.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_uint64, _u8p, _u8p,
                                ctypes.c_size_t]
        lib.ref_cbc.restype = ctypes.c_int
        lib.ref_cbc.argtypes = [ctypes.c_int, _u8p, ctypes.c_int, _u8p, _u8p, _u8p, ctypes.c_size_t]
        lib.ref_xts_mul_alpha.argtypes = [_u8p]
        lib.ref_xts.restype = ctypes.c_int
        lib.ref_xts.argtypes = [ctypes.c_int, _u8p, _u8p, ctypes.c_int, ctypes.c_size_t, ctypes.c_uint64,
                                _u8p, _u8p, ctypes.c_size_t]
        lib.ref_gcm_mul.argtypes = [_u8p, _u8p, _u8p]
        lib.ref_ghash.argtypes = [_u8p, _u8p, ctypes.c_size_t, _u8p]
        lib.ref_gcm_j0.argtypes = [_u8p, _u8p, ctypes.c_size_t, _u8p]
        lib.ref_gcm_encrypt.restype = ctypes.c_int
        lib.ref_gcm_encrypt.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_size_t, _u8p, ctypes.c_size_t,
                                        _u8p, _u8p, ctypes.c_size_t, _u8p]
        lib.ref_gcm_decrypt.restype = ctypes.c_int
        lib.ref_gcm_decrypt.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_size_t, _u8p, ctypes.c_size_t,
                                        _u8p, _u8p, ctypes.c_size_t, _u8p, ctypes.c_size_t]
        lib.ref_par_run.restype = ctypes.c_int
        lib.ref_par_run.argtypes = [ctypes.c_int, _u8p, ctypes.c_int, _u8p, _u8p, _u8p,
                                    ctypes.c_size_t, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double)]
        self.lib = lib
        self.path = path

    # --- GF(2^8) and tables -------------------------------------------------
    def xtime(self, b):
        return self.lib.ref_xtime(b)

    def gf_mul(self, a, b):
        return self.lib.ref_gf_mul(a, b)

    def rcon(self, j):
        return self.lib.ref_rcon(j)

    def sbox(self):
        out = np.zeros(256, np.uint8)
        self.lib.ref_sbox(_ptr(out))
        return out

    def inv_sbox(self):
        out = np.zeros(256, np.uint8)
        self.lib.ref_inv_sbox(_ptr(out))
        return out

    def step(self, name, block):
        """Apply one named transformation to a 16-byte block (column order)."""
        b = _as_u8(block).copy()
        assert b.size == 16
        getattr(self.lib, "ref_step_" + name)(_ptr(b))
        return b

    # --- key schedule and block cipher ----------------------------------
    def expand_key(self, key):
        """Returns (round key bytes, Nr) for a 16-, 24- or 32-byte key."""
        k = _as_u8(key)
        w = np.zeros(240, np.uint8)
        nr = self.lib.ref_expand_key(_ptr(k), 8 * k.size, _ptr(w))
        if nr < 0:
            raise ValueError("unsupported key length %d bytes" % k.size)
        return w[:16 * (nr + 1)].copy(), nr

    def encrypt_block(self, rk, nr, block):
        b, out = _as_u8(block), np.zeros(16, np.uint8)
        self.lib.ref_encrypt_block(_ptr(_as_u8(rk)), nr, _ptr(b), _ptr(out))
        return out

    def decrypt_block(self, rk, nr, block):
        b, out = _as_u8(block), np.zeros(16, np.uint8)
        self.lib.ref_decrypt_block(_ptr(_as_u8(rk)), nr, _ptr(b), _ptr(out))
        return out

    # --- modes ----------------------------------------------------------
    def ecb(self, decrypt, rk, nr, data):
        d = _as_u8(data)
        out = np.empty_like(d)
        if self.lib.ref_ecb(1 if decrypt else 0, _ptr(_as_u8(rk)), nr, _ptr(d), _ptr(out), d.size):
            raise ValueError("ECB length must be a multiple of 16")
        return out

    def ecb_encrypt(self, rk, nr, data):
        return self.ecb(False, rk, nr, data)

    def ecb_decrypt(self, rk, nr, data):
        return self.ecb(True, rk, nr, data)

    def ctr_block(self, ctr0, j):
        out = np.zeros(16, np.uint8)
        self.lib.ref_ctr_block(_ptr(_as_u8(ctr0)), j, _ptr(out))
        return out

    def ctr(self, rk, nr, ctr0, data, first_block=0):
        d = _as_u8(data)
        out = np.empty_like(d)
        self.lib.ref_ctr(_ptr(_as_u8(rk)), nr, _ptr(_as_u8(ctr0)), first_block, _ptr(d),
                         _ptr(out), d.size)
        return out

    def cbc(self, decrypt, rk, nr, iv, data):
        d = _as_u8(data)
        out = np.empty_like(d)
        if self.lib.ref_cbc(1 if decrypt else 0, _ptr(_as_u8(rk)), nr, _ptr(_as_u8(iv)), _ptr(d),
                            _ptr(out), d.size):
            raise ValueError("CBC length must be a multiple of 16")
        return out

    def cbc_encrypt(self, rk, nr, iv, data):
        return self.cbc(False, rk, nr, iv, data)

    def cbc_decrypt(self, rk, nr, iv, data):
        return self.cbc(True, rk, nr, iv, data)

    def xts_mul_alpha(self, t):
        b = _as_u8(t).copy()
        self.lib.ref_xts_mul_alpha(_ptr(b))
        return b

    def xts(self, decrypt, rk1, rk2, nr, unit_bytes, first_unit, data):
        d = _as_u8(data)
        out = np.empty_like(d)
        if self.lib.ref_xts(1 if decrypt else 0, _ptr(_as_u8(rk1)), _ptr(_as_u8(rk2)), nr, unit_bytes,
                            first_unit, _ptr(d), _ptr(out), d.size):
            raise ValueError("XTS lengths must be multiples of 16")
        return out

    def gcm_mul(self, x, y):
        """Product in GF(2^128), the GCM bit order."""
        out = np.zeros(16, np.uint8)
        self.lib.ref_gcm_mul(_ptr(_as_u8(x)), _ptr(_as_u8(y)), _ptr(out))
        return out

    def ghash(self, h, data, y=None):
        """GHASH_H over whole blocks of `data`, continuing from `y` (zero)."""
        d = _as_u8(data)
        assert d.size % 16 == 0
        out = np.zeros(16, np.uint8) if y is None else _as_u8(y).copy()
        self.lib.ref_ghash(_ptr(_as_u8(h)), _ptr(d) if d.size else None, d.size // 16, _ptr(out))
        return out

    def gcm_j0(self, h, iv):
        v = _as_u8(iv)
        out = np.zeros(16, np.uint8)
        self.lib.ref_gcm_j0(_ptr(_as_u8(h)), _ptr(v), v.size, _ptr(out))
        return out

    def gcm_encrypt(self, rk, nr, iv, aad, data):
        """Returns (ciphertext, 16-byte tag)."""
        v, a, d = _as_u8(iv), _as_u8(aad), _as_u8(data)
        out, tag = np.empty_like(d), np.zeros(16, np.uint8)
        if self.lib.ref_gcm_encrypt(_ptr(_as_u8(rk)), nr, _ptr(v), v.size, _ptr(a) if a.size else None,
                                    a.size, _ptr(d) if d.size else None, _ptr(out) if d.size else None,
                                    d.size, _ptr(tag)):
            raise ValueError("GCM needs a non-empty IV")
        return out, tag

    def gcm_decrypt(self, rk, nr, iv, aad, data, tag):
        """Returns (plaintext, authentic?) for the given (possibly truncated) tag."""
        v, a, d, t = _as_u8(iv), _as_u8(aad), _as_u8(data), _as_u8(tag)
        out = np.empty_like(d)
        rc = self.lib.ref_gcm_decrypt(_ptr(_as_u8(rk)), nr, _ptr(v), v.size, _ptr(a) if a.size else None,
                                      a.size, _ptr(d) if d.size else None, _ptr(out) if d.size else None,
                                      d.size, _ptr(t), t.size)
        if rc < 0:
            raise ValueError("GCM needs a non-empty IV and a tag of 1..16 bytes")
        return out, rc == 0

    def par_run(self, op, rk, nr, data, nthreads, ctr0=None, out=None):
        """The paper's pthreads method; returns (output, seconds)."""
        d = _as_u8(data)
        if out is None:
            out = np.empty_like(d)
        c0 = _as_u8(ctr0) if ctr0 is not None else np.zeros(16, np.uint8)
        secs = ctypes.c_double(0.0)
        rc = self.lib.ref_par_run(op, _ptr(_as_u8(rk)), nr, _ptr(c0), _ptr(d), _ptr(out),
                                  d.size, nthreads, ctypes.byref(secs))
        if rc:
            raise ValueError("ref_par_run rejected its arguments")
        return out, secs.value


_default = None


def default():
    """The oracle built from the sources as committed (no planted mistakes)."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
