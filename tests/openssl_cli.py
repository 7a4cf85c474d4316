"""Runs the system's ``openssl enc`` executable as an independent AES.

The executable is only run on inputs and its output compared; nothing of it
is read or linked.  Its CTR mode increments the whole 128-bit counter block,
so callers compare against it only on ranges where the low 32-bit counter
does not wrap (there the two counting rules agree).
"""
import shutil
import subprocess

import numpy as np

OPENSSL = shutil.which("openssl")


def available():
    if OPENSSL is None:
        return False
    r = subprocess.run([OPENSSL, "enc", "-aes-128-ecb", "-nopad", "-K", "00" * 16],
                       input=b"\0" * 16, capture_output=True)
    return r.returncode == 0 and len(r.stdout) == 16


def enc(mode, key, data, iv=None, decrypt=False):
    """``openssl enc -aes-<bits>-<mode>`` on `data`; returns numpy uint8."""
    key = bytes(np.asarray(key, dtype=np.uint8))
    cmd = [OPENSSL, "enc", "-aes-%d-%s" % (8 * len(key), mode), "-K", key.hex()]
    if mode in ("ecb", "cbc"):
        cmd.append("-nopad")
    if iv is not None:
        cmd += ["-iv", bytes(np.asarray(iv, dtype=np.uint8)).hex()]
    if decrypt:
        cmd.append("-d")
    r = subprocess.run(cmd, input=bytes(np.asarray(data, dtype=np.uint8)),
                       capture_output=True, check=True)
    return np.frombuffer(r.stdout, dtype=np.uint8).copy()


def gmac(key, iv, data):
    """``openssl mac -cipher AES-<bits>-GCM ... GMAC``: the GCM tag of an
    empty plaintext with `data` as the additional authenticated data."""
    key = bytes(np.asarray(key, dtype=np.uint8))
    iv = bytes(np.asarray(iv, dtype=np.uint8))
    cmd = [OPENSSL, "mac", "-cipher", "AES-%d-GCM" % (8 * len(key)), "-macopt", "hexkey:" + key.hex(),
           "-macopt", "hexiv:" + iv.hex(), "GMAC"]
    data = bytes(data) if isinstance(data, (bytes, bytearray)) else bytes(np.asarray(data, dtype=np.uint8))
    r = subprocess.run(cmd, input=data, capture_output=True, check=True)
    return np.frombuffer(bytes.fromhex(r.stdout.decode().strip()), dtype=np.uint8).copy()
