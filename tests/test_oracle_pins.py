"""The oracle against its pins (mathematics of AES and an independent AES).

A failure here means the oracle itself is wrong; nothing else can be trusted
until these pass.
"""
import numpy as np
import pytest

import seedgen
from oracle import ref
from tests import libcrypto_evp, openssl_cli, pins


@pytest.fixture(scope="module")
def o():
    return ref.default()


def test_gf_arithmetic(o):
    assert pins.pin_gf(o) == []


def test_sbox_closed_form_and_structure(o):
    assert pins.pin_sbox(o) == []


def test_mix_columns_polynomial_and_inverse(o):
    assert pins.pin_mix_columns(o) == []


def test_shift_rows(o):
    assert pins.pin_shift_rows(o) == []


def test_key_expansion_prefix(o):
    assert pins.pin_key_expansion(o) == []


@pytest.mark.skipif(not openssl_cli.available(), reason="openssl executable not present")
def test_against_openssl_executable(o):
    # 3 key sizes x 8 keys x 128 blocks = 3072 (key, block) pairs per direction
    assert pins.pin_openssl(o) == []


@pytest.mark.skipif(not openssl_cli.available(), reason="openssl executable not present")
def test_against_openssl_1mib(o):
    k = seedgen.key(2, 0, 128)
    w, nr = o.expand_key(k)
    pt = seedgen.data_np(2, 0, 1 << 20)
    assert np.array_equal(o.ecb_encrypt(w, nr, pt), openssl_cli.enc("ecb", k, pt))
    ctr0 = seedgen.nonce(2, 0)
    assert np.array_equal(o.ctr(w, nr, ctr0, pt), openssl_cli.enc("ctr", k, pt, iv=ctr0))


def test_ctr_structure(o):
    assert pins.pin_ctr_structure(o) == []


def test_roundtrip(o):
    assert pins.pin_roundtrip(o) == []


def test_chunking_premise(o):
    assert pins.pin_chunking(o) == []


def test_bad_arguments(o):
    with pytest.raises(ValueError):
        o.expand_key(np.zeros(20, np.uint8))
    w, nr = o.expand_key(np.zeros(16, np.uint8))
    with pytest.raises(ValueError):
        o.ecb_encrypt(w, nr, np.zeros(17, np.uint8))
    with pytest.raises(ValueError):
        o.par_run(0, w, nr, np.zeros(17, np.uint8), 2)


def test_cbc(o):
    assert pins.pin_cbc(o) == []


def test_xts(o):
    assert pins.pin_xts(o) == []


def test_gcm(o):
    assert pins.pin_gcm(o) == []


@pytest.mark.skipif(not libcrypto_evp.available(b"AES-128-XTS"), reason="libcrypto AES-XTS not present")
def test_xts_against_libcrypto(o):
    assert pins.pin_xts_evp(o) == []


@pytest.mark.skipif(not libcrypto_evp.available(b"AES-128-GCM"), reason="libcrypto AES-GCM not present")
def test_gcm_against_libcrypto(o):
    assert pins.pin_gcm_evp(o) == []


def test_gf128_reference_is_a_field_multiplication():
    # the test-side GF(2^128) itself: commutative, distributive, x * x^127 = x^128
    import random
    rnd = random.Random(5)
    for _ in range(20):
        a, b, c = (rnd.getrandbits(128) for _ in range(3))
        assert pins.gf128_mul_int(a, b) == pins.gf128_mul_int(b, a)
        assert pins.gf128_mul_int(a, b ^ c) == pins.gf128_mul_int(a, b) ^ pins.gf128_mul_int(a, c)
    assert pins.gf128_mul_int(2, 1 << 127) == 0x87
    t = rnd.getrandbits(128)
    x = t
    for _ in range(37):
        x = pins.gf128_mulx_int(x)
    assert x == pins.gf128_mul_int(t, 1 << 37)
