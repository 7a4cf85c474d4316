"""The C ABI from plain C: tests/cpp/abi_client (built with the library)
calls aes_expand_key, aes_encrypt/aes_decrypt (ECB, CTR), aes_xts_* and
aes_gcm_* with device memory from the HIP runtime alone; its outputs must
equal the oracle's byte for byte."""
import os
import struct
import subprocess

import numpy as np
import pytest

import seedgen
from oracle import ref

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cpp", "abi_client")

CASES = [(128, 100003, 33, 512, 7), (256, (1 << 20) + 16, 0, 4096, (1 << 40) + 3), (192, 0, 64, 16, 0),
         (128, 4096 * 70 + 48, 16, 4096, 123)]


@pytest.mark.parametrize("bits,nbytes,aad_bytes,unit,first", CASES,
                         ids=["%d-%d-%d-%d" % c[:4] for c in CASES])
def test_c_client_matches_oracle(tmp_path, bits, nbytes, aad_bytes, unit, first):
    assert os.path.exists(EXE), "tests/cpp/abi_client is not built (the package build builds it)"
    o = ref.default()
    key = np.zeros(32, np.uint8)
    key2 = np.zeros(32, np.uint8)
    key[:bits // 8] = seedgen.key(60, nbytes % 997, bits)
    key2[:bits // 8] = seedgen.key(61, nbytes % 997, bits)
    ctr0 = seedgen.nonce(60, bits)
    aad = seedgen.data_np(62, aad_bytes, aad_bytes)
    data = seedgen.data_np(63, nbytes % 1013, nbytes)
    job = os.path.join(str(tmp_path), "job.bin")
    out = os.path.join(str(tmp_path), "out.bin")
    with open(job, "wb") as f:
        f.write(key.tobytes() + key2.tobytes() + struct.pack("<IIQ", bits, unit, first) + ctr0.tobytes() +
                struct.pack("<IQ", aad_bytes, nbytes) + aad.tobytes() + data.tobytes())
    r = subprocess.run([EXE, job, out], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    res = np.fromfile(out, dtype=np.uint8)
    n16 = nbytes // 16 * 16
    parts, at = [], 0
    for ln in (n16, nbytes, n16, nbytes, 16, 16):
        parts.append(res[at:at + ln])
        at += ln
    assert at == res.size
    ecb, ctr, xts, gcm, tag, status = parts
    rk, nr = o.expand_key(key[:bits // 8])
    rk2, _ = o.expand_key(key2[:bits // 8])
    assert np.array_equal(ecb, o.ecb_encrypt(rk, nr, data[:n16]))
    assert np.array_equal(ctr, o.ctr(rk, nr, ctr0, data))
    assert np.array_equal(xts, o.xts(False, rk, rk2, nr, unit, first, data[:n16]))
    want_ct, want_tag = o.gcm_encrypt(rk, nr, ctr0[:12], aad, data)
    assert np.array_equal(gcm, want_ct)
    assert np.array_equal(tag, want_tag)
    verdict_ok, verdict_bad, ecb_back, xts_back = struct.unpack("<4i", status.tobytes())
    assert (verdict_ok, verdict_bad, ecb_back, xts_back) == (1, 0, 1, 1)
