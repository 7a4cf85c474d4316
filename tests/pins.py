"""Pins for the oracle: checks against facts fixed by the mathematics of
AES and by an independent AES (the openssl executable), never against the
oracle's own formulas.

Each function takes an ``oracle.ref.Oracle`` and returns a list of failure
strings (empty when the pin holds), so that the same pins run both on the
oracle as committed and on copies with a planted mistake, where at least one
of them must fail.
"""
import numpy as np

import seedgen
from tests import libcrypto_evp, openssl_cli

POLY = 0x11B  # x^8 + x^4 + x^3 + x + 1


# --- an independent GF(2^8): carry-less product, then long division -------
def clmul(a, b):
    p = 0
    for i in range(8):
        if (b >> i) & 1:
            p ^= a << i
    return p


def reduce_poly(p):
    for bit in range(14, 7, -1):
        if (p >> bit) & 1:
            p ^= POLY << (bit - 8)
    return p


def gmul(a, b):
    return reduce_poly(clmul(a, b))


def gpow(a, e):
    r = 1
    for _ in range(e):
        r = gmul(r, a)
    return r


def rotl8(b, n):
    return ((b << n) | (b >> (8 - n))) & 0xFF


def sbox_closed_form(x):
    """S(x) = A(x^254) + 0x63 with A as the circulant sum of rotations."""
    inv = gpow(x, 254)  # x^254 = x^-1 for x != 0, and 0 for x = 0
    return inv ^ rotl8(inv, 1) ^ rotl8(inv, 2) ^ rotl8(inv, 3) ^ rotl8(inv, 4) ^ 0x63


def poly_mulmod4(a, col):
    """(a0 + a1 x + a2 x^2 + a3 x^3) * col(x) mod x^4 + 1, coefficients in GF(2^8)."""
    out = [0, 0, 0, 0]
    for i in range(4):
        for j in range(4):
            out[(i + j) % 4] ^= gmul(a[i], col[j])
    return out


MIX_POLY = (0x02, 0x01, 0x01, 0x03)      # a(x) = {03}x^3 + {01}x^2 + {01}x + {02}
INV_MIX_POLY = (0x0E, 0x09, 0x0D, 0x0B)  # a^-1(x) = {0b}x^3 + {0d}x^2 + {09}x + {0e}


# --- pins -----------------------------------------------------------------
def pin_gf(o):
    fails = []
    for a in range(256):
        if o.xtime(a) != gmul(a, 2):
            fails.append("xtime(%#x)" % a)
            break
    for a in range(256):
        for b in range(256):
            if o.gf_mul(a, b) != gmul(a, b):
                fails.append("gf_mul(%#x,%#x)" % (a, b))
                return fails
    for j in range(1, 15):
        if o.rcon(j) != gpow(2, j - 1):
            fails.append("rcon[%d]" % j)
    return fails


def pin_sbox(o):
    fails = []
    s, inv = o.sbox(), o.inv_sbox()
    expect = np.array([sbox_closed_form(x) for x in range(256)], np.uint8)
    if not np.array_equal(s, expect):
        fails.append("sbox != closed form at %s" % np.nonzero(s != expect)[0][:4])
    if len(set(s.tolist())) != 256:
        fails.append("sbox not a bijection")
    if not np.array_equal(inv[s], np.arange(256, dtype=np.uint8)):
        fails.append("inv_sbox . sbox != id")
    x = np.arange(256)
    if np.any(s == x) or np.any(s == (x ^ 0xFF)):
        fails.append("sbox has a fixed or opposite-fixed point")
    blk = seedgen.bytes_np(seedgen.stream_seed(7, seedgen.TAG_DATA), 16)
    if not np.array_equal(o.step("sub_bytes", blk), s[blk]):
        fails.append("SubBytes step != sbox per byte")
    return fails


def _cols(block):
    return [list(block[4 * c:4 * c + 4]) for c in range(4)]


def pin_mix_columns(o):
    """MixColumns is GF(2)-linear, so agreement with the polynomial product on
    all 128 single-bit states, plus linearity, fixes it completely."""
    fails = []
    for name, poly in (("mix_columns", MIX_POLY), ("inv_mix_columns", INV_MIX_POLY)):
        for bit in range(128):
            b = np.zeros(16, np.uint8)
            b[bit // 8] = 1 << (bit % 8)
            got = o.step(name, b)
            want = np.array(sum((poly_mulmod4(poly, c) for c in _cols(b)), []), np.uint8)
            if not np.array_equal(got, want):
                fails.append("%s on basis bit %d" % (name, bit))
                break
        rnd = seedgen.bytes_np(seedgen.stream_seed(11, seedgen.TAG_DATA), 32 * 16).reshape(-1, 16)
        for i in range(0, len(rnd), 2):
            x, y = rnd[i], rnd[i + 1]
            if not np.array_equal(o.step(name, x ^ y), o.step(name, x) ^ o.step(name, y)):
                fails.append("%s not linear" % name)
                break
    rnd = seedgen.bytes_np(seedgen.stream_seed(12, seedgen.TAG_DATA), 16 * 16).reshape(-1, 16)
    for x in rnd:
        if not np.array_equal(o.step("inv_mix_columns", o.step("mix_columns", x)), x):
            fails.append("InvMixColumns . MixColumns != id")
            break
    return fails


def pin_shift_rows(o):
    """Row r of the 4x4 state (s[r][c] = in[r + 4c]) rotates left by r."""
    fails = []
    b = np.arange(16, dtype=np.uint8)
    m = b.reshape(4, 4).T          # m[r][c] = b[r + 4c]
    want = np.stack([np.roll(m[r], -r) for r in range(4)]).T.reshape(-1)
    if not np.array_equal(o.step("shift_rows", b), want):
        fails.append("ShiftRows permutation")
    if not np.array_equal(o.step("inv_shift_rows", o.step("shift_rows", b)), b):
        fails.append("InvShiftRows . ShiftRows != id")
    return fails


def pin_key_expansion(o):
    fails = []
    for bits in (128, 192, 256):
        k = seedgen.key(21, bits, bits)
        w, nr = o.expand_key(k)
        if nr != bits // 32 + 6 or w.size != 16 * (nr + 1):
            fails.append("AES-%d: Nr/length" % bits)
        if not np.array_equal(w[:bits // 8], k):
            fails.append("AES-%d: first Nk words != key" % bits)
    return fails


def pin_openssl(o, nkeys=8, blocks_per_key=128):
    """Whole-cipher agreement with an independent AES (the openssl
    executable): ECB both ways for every key size, CTR with tails."""
    if not openssl_cli.available():
        return ["openssl executable not available"]
    fails = []
    for bits in (128, 192, 256):
        for i in range(nkeys):
            k = seedgen.key(31, 1000 * bits + i, bits)
            w, nr = o.expand_key(k)
            pt = seedgen.data_np(31, 1000 * bits + i, 16 * blocks_per_key)
            ct = o.ecb_encrypt(w, nr, pt)
            if not np.array_equal(ct, openssl_cli.enc("ecb", k, pt)):
                fails.append("ECB-%d encrypt, key %d" % (bits, i))
                break
            if not np.array_equal(o.ecb_decrypt(w, nr, pt), openssl_cli.enc("ecb", k, pt, decrypt=True)):
                fails.append("ECB-%d decrypt, key %d" % (bits, i))
                break
            n = 16 * blocks_per_key - 16 + 1 + (i * 5) % 15   # partial final block
            ctr0 = seedgen.nonce(31, 1000 * bits + i)
            got = o.ctr(w, nr, ctr0, pt[:n])
            if not np.array_equal(got, openssl_cli.enc("ctr", k, pt[:n], iv=ctr0)):
                fails.append("CTR-%d, key %d, %d bytes" % (bits, i, n))
                break
    return fails


def pin_ctr_structure(o):
    """CTR keystream block j is Cipher(T_j) with T_j = nonce || BE32(c0+j),
    the counter wraps modulo 2^32 without carrying into the nonce, a partial
    tail is a prefix of the full-block result, and CTR is an involution."""
    fails = []
    k = seedgen.key(41, 0, 128)
    w, nr = o.expand_key(k)
    ctr0 = seedgen.nonce(41, 0)
    ctr0[12:16] = [0xFF, 0xFF, 0xFF, 0xF0]        # counter wraps after 16 blocks
    zeros = np.zeros(16 * 40, np.uint8)
    ks = o.ctr(w, nr, ctr0, zeros)
    for j in range(40):
        c = (0xFFFFFFF0 + j) & 0xFFFFFFFF
        t = np.concatenate([ctr0[:12], np.array([c >> 24, (c >> 16) & 255, (c >> 8) & 255, c & 255], np.uint8)])
        if not np.array_equal(o.ctr_block(ctr0, j), t):
            fails.append("counter block %d layout" % j)
            break
        if not np.array_equal(ks[16 * j:16 * j + 16], o.encrypt_block(w, nr, t)):
            fails.append("keystream block %d != Cipher(T_j)" % j)
            break
    pt = seedgen.data_np(41, 1, 16 * 40)
    full = o.ctr(w, nr, ctr0, pt)
    for n in (0, 1, 15, 17, 33, 16 * 40 - 1):
        if not np.array_equal(o.ctr(w, nr, ctr0, pt[:n]), full[:n]):
            fails.append("CTR tail of %d bytes is not a prefix" % n)
    if not np.array_equal(o.ctr(w, nr, ctr0, full), pt):
        fails.append("CTR is not an involution")
    return fails


def pin_roundtrip(o):
    fails = []
    for bits in (128, 192, 256):
        k = seedgen.key(51, bits, bits)
        w, nr = o.expand_key(k)
        pt = seedgen.data_np(51, bits, 16 * 64)
        if not np.array_equal(o.ecb_decrypt(w, nr, o.ecb_encrypt(w, nr, pt)), pt):
            fails.append("AES-%d: decrypt(encrypt(x)) != x" % bits)
    return fails


def pin_chunking(o):
    """The paper's premise: chunks processed apart and concatenated equal the
    whole (checked through the pthreads runner)."""
    fails = []
    k = seedgen.key(61, 0, 256)
    w, nr = o.expand_key(k)
    ctr0 = seedgen.nonce(61, 0)
    pt = seedgen.data_np(61, 0, 16 * 1000 + 9)
    whole_ecb = o.ecb_encrypt(w, nr, pt[:16 * 1000])
    whole_ctr = o.ctr(w, nr, ctr0, pt)
    for t in (1, 2, 3, 7, 32, 64):
        got, _ = o.par_run(0, w, nr, pt[:16 * 1000], t)
        if not np.array_equal(got, whole_ecb):
            fails.append("ECB with %d chunks" % t)
        got, _ = o.par_run(2, w, nr, pt, t, ctr0=ctr0)
        if not np.array_equal(got, whole_ctr):
            fails.append("CTR with %d chunks" % t)
    return fails


def pin_cbc(o, nkeys=4, blocks=64):
    """CBC against the openssl executable, both directions, every key size,
    plus decrypt(encrypt(x)) = x and the structure of the chaining: flipping
    one ciphertext bit garbles that block and flips the same bit of the next
    plaintext block only."""
    fails = []
    have_openssl = openssl_cli.available()
    for bits in (128, 192, 256):
        for i in range(nkeys):
            k = seedgen.key(71, 100 * bits + i, bits)
            w, nr = o.expand_key(k)
            iv = seedgen.bytes_np(seedgen.stream_seed(71, seedgen.TAG_NONCE, 100 * bits + i), 16)
            pt = seedgen.data_np(71, 100 * bits + i, 16 * blocks)
            ct = o.cbc_encrypt(w, nr, iv, pt)
            if have_openssl:
                if not np.array_equal(ct, openssl_cli.enc("cbc", k, pt, iv=iv)):
                    fails.append("CBC-%d encrypt vs openssl, key %d" % (bits, i))
                    break
                if not np.array_equal(o.cbc_decrypt(w, nr, iv, pt), openssl_cli.enc("cbc", k, pt, iv=iv, decrypt=True)):
                    fails.append("CBC-%d decrypt vs openssl, key %d" % (bits, i))
                    break
            if not np.array_equal(o.cbc_decrypt(w, nr, iv, ct), pt):
                fails.append("CBC-%d decrypt(encrypt(x)) != x" % bits)
            bad = ct.copy()
            bad[16 * 5 + 3] ^= 0x10
            d = o.cbc_decrypt(w, nr, iv, bad)
            diff = np.nonzero(d != pt)[0]
            if not (diff.min() >= 16 * 5 and diff.max() < 16 * 7 and d[16 * 6 + 3] == pt[16 * 6 + 3] ^ 0x10
                    and (d[16 * 6:16 * 7] != pt[16 * 6:16 * 7]).sum() == 1):
                fails.append("CBC-%d error propagation" % bits)
    return fails


# --- an independent GF(2^128) for XTS: Python integers ---------------------
XTS_POLY = (1 << 128) | 0x87          # x^128 + x^7 + x^2 + x + 1


def gf128_mulx_int(t):
    t <<= 1
    return t ^ XTS_POLY if t >> 128 else t


def gf128_mul_int(a, b):
    """Carry-less product reduced by the XTS polynomial (bit k = x^k)."""
    p = 0
    for k in range(128):
        if (b >> k) & 1:
            p ^= a << k
    for k in range(254, 127, -1):
        if (p >> k) & 1:
            p ^= XTS_POLY << (k - 128)
    return p


def pin_xts(o):
    """XTS rebuilt block by block from pinned pieces: T_j from the ECB
    encryption (pinned against openssl) of the little-endian unit number and
    an independent GF(2^128) (Python integers: x^j by repeated doubling, and
    by a general carry-less product with x^j), each block through ECB.  The
    conventions themselves (tweak byte order, placement of alpha^j) are
    pinned against an independent XTS by pin_xts_evp."""
    fails = []
    for k in range(200):
        t = int.from_bytes(seedgen.bytes_np(seedgen.stream_seed(81, seedgen.TAG_DATA, k), 16).tobytes(), "little")
        want = gf128_mulx_int(t).to_bytes(16, "little")
        got = bytes(o.xts_mul_alpha(np.frombuffer(t.to_bytes(16, "little"), np.uint8)))
        if got != want:
            fails.append("alpha multiplication")
            break
    for bits in (128, 256):
        k1, k2 = seedgen.key(82, bits, bits), seedgen.key(82, bits + 1, bits)
        w1, nr = o.expand_key(k1)
        w2, _ = o.expand_key(k2)
        for unit, nblocks, first in ((512, 80, 7), (4096, 300, 1 << 40), (16, 5, 0)):
            pt = seedgen.data_np(82, unit + bits, 16 * nblocks)
            ct = o.xts(False, w1, w2, nr, unit, first, pt)
            want = np.empty_like(pt)
            for j in range(nblocks):
                u, jj = divmod(16 * j, unit)
                iv = np.frombuffer((first + u).to_bytes(16, "little"), np.uint8)
                t0 = int.from_bytes(o.encrypt_block(w2, nr, iv).tobytes(), "little")
                e = jj // 16
                # x^e: a general product for e < 128, repeated doubling beyond
                tj = gf128_mul_int(t0, 1 << e) if e < 128 else t0
                for _ in range(e if e >= 128 else 0):
                    tj = gf128_mulx_int(tj)
                tb = np.frombuffer(tj.to_bytes(16, "little"), np.uint8)
                want[16 * j:16 * j + 16] = o.encrypt_block(w1, nr, pt[16 * j:16 * j + 16] ^ tb) ^ tb
            if not np.array_equal(ct, want):
                fails.append("XTS-%d unit %d" % (bits, unit))
            if not np.array_equal(o.xts(True, w1, w2, nr, unit, first, ct), pt):
                fails.append("XTS-%d decrypt(encrypt(x)) != x" % bits)
    return fails


def pin_xts_evp(o):
    """XTS against an independent implementation, libcrypto's EVP AES-XTS
    (called, never read).  Each data unit goes through EVP with key K1 || K2
    and the tweak block = the unit's sequence number as a 16-byte
    little-endian number (IEEE 1619's encoding of the data-unit sequence
    number); the oracle runs the whole buffer in one call.  Units of 16 B to
    4 KiB, a shorter last unit, sequence numbers across 2^32 and up to the
    wrap at 2^64, both directions.  This pins the tweak's byte order and
    where alpha^j enters, which pin_xts only restates."""
    fails = []
    if not (libcrypto_evp.available(b"AES-128-XTS") and libcrypto_evp.available(b"AES-256-XTS")):
        return ["libcrypto AES-XTS not available"]
    cases = ((16, 7, 0), (32, 9, 123456789), (512, 70, (1 << 32) - 2), (4096, 600, 5),
             (4096, 300, (1 << 64) - 1), (512, 33, (1 << 64) - 5), (1024, 200, 1 << 40))
    for bits in (128, 256):
        k1, k2 = seedgen.key(83, bits, bits), seedgen.key(83, bits + 1, bits)
        w1, nr = o.expand_key(k1)
        w2, _ = o.expand_key(k2)
        for ci, (unit, nblocks, first) in enumerate(cases):
            data = seedgen.data_np(83, 1000 * bits + ci, 16 * nblocks)
            for decrypt in (False, True):
                got = o.xts(decrypt, w1, w2, nr, unit, first, data)
                want = np.empty_like(data)
                for u0 in range(0, data.size, unit):
                    tweak = ((first + u0 // unit) % (1 << 64)).to_bytes(16, "little")
                    seg = data[u0:u0 + unit]
                    want[u0:u0 + seg.size] = libcrypto_evp.xts_unit(k1, k2, tweak, seg, decrypt)
                if not np.array_equal(got, want):
                    fails.append("XTS-%d %s, unit %d, first unit %d" % (bits, "dec" if decrypt else "enc",
                                                                         unit, first))
    return fails


def pin_gcm_evp(o):
    """GCM against an independent implementation, libcrypto's EVP AES-GCM
    (called, never read): ciphertext and full tag for 128-, 192- and 256-bit
    keys, IVs of 1 .. 128 bytes (libcrypto takes at most 128), additional
    data and plaintext of 0 .. 1000 bytes with partial last blocks;
    decryption's plaintext and verdict for the tag, truncated tags and a
    changed tag."""
    fails = []
    if not all(libcrypto_evp.available(n) for n in (b"AES-128-GCM", b"AES-192-GCM", b"AES-256-GCM")):
        return ["libcrypto AES-GCM not available"]
    shapes = ((12, 0, 0), (12, 16, 64), (12, 45, 1000), (1, 7, 33), (13, 0, 16), (16, 1, 15),
              (60, 1000, 5), (128, 17, 16 * 37))
    for bits in (128, 192, 256):
        for si, (ivlen, alen, plen) in enumerate(shapes):
            key = seedgen.key(97, 100 * bits + si, bits)
            w, nr = o.expand_key(key)
            iv = seedgen.bytes_np(seedgen.stream_seed(97, seedgen.TAG_NONCE, 1000 * bits + si), ivlen)
            aad = seedgen.data_np(98, 1000 * bits + si, alen)
            pt = seedgen.data_np(99, 1000 * bits + si, plen)
            ct, tag = o.gcm_encrypt(w, nr, iv, aad, pt)
            ect, etag = libcrypto_evp.gcm_encrypt(key, iv, aad, pt)
            if not np.array_equal(ct, ect) or not np.array_equal(tag, etag):
                fails.append("GCM-%d encrypt, IV %d B, AAD %d B, %d B" % (bits, ivlen, alen, plen))
                continue
            for tlen in (16, 12, 8, 4):
                back, ok = o.gcm_decrypt(w, nr, iv, aad, ct, etag[:tlen])
                eback, eok = libcrypto_evp.gcm_decrypt(key, iv, aad, ct, etag[:tlen])
                if not (ok and eok and np.array_equal(back, eback) and np.array_equal(back, pt)):
                    fails.append("GCM-%d decrypt, %d-byte tag" % (bits, tlen))
            bad = etag.copy()
            bad[-1] ^= 0x01
            if o.gcm_decrypt(w, nr, iv, aad, ct, bad)[1] or libcrypto_evp.gcm_decrypt(key, iv, aad, ct, bad)[1]:
                fails.append("GCM-%d changed tag accepted" % bits)
    return fails


def gcm_to_int(b):
    """A block in GCM's bit order (bit 0 = most significant bit of byte 0 =
    coefficient of x^0) as an integer whose bit i is the coefficient of x^i:
    the bits of every byte reversed, bytes little-endian."""
    return int.from_bytes(bytes(int("{:08b}".format(x)[::-1], 2) for x in bytes(b)), "little")


def int_to_gcm(v):
    return np.frombuffer(bytes(int("{:08b}".format(x)[::-1], 2) for x in v.to_bytes(16, "little")), np.uint8)


def gcm_mul_int(a, b):
    # GCM reduces by the same x^128 + x^7 + x^2 + x + 1 as XTS; only the bit order differs
    return int_to_gcm(gf128_mul_int(gcm_to_int(a), gcm_to_int(b)))


def _be64(v):
    return v.to_bytes(8, "big")


def pin_gcm(o, nkeys=2):
    """GCM from pieces pinned elsewhere:
    - the GF(2^128) product against an independent carry-less product;
    - tags of empty plaintexts against the openssl executable's GMAC (which
      is GCM with the message as additional data), for IVs of 12 and of
      other lengths (the GHASH-derived pre-counter block);
    - the ciphertext against openssl CTR started one past the pre-counter
      block J0, where Cipher(J0) is read off openssl's GMAC of an empty
      message and J0 = InvCipher of it (openssl ECB);
    - tags with a plaintext through GHASH's linearity: with additional data
      of whole blocks, tag(A, C) = GMAC(A || C padded) XOR (L1 XOR L2) * H,
      L1, L2 the two length blocks and H = Cipher(0) (openssl ECB);
    - decryption accepts the tag, a truncated tag, and rejects any change."""
    fails = []
    for k in range(300):
        a = seedgen.bytes_np(seedgen.stream_seed(91, seedgen.TAG_DATA, 2 * k), 16)
        b = seedgen.bytes_np(seedgen.stream_seed(91, seedgen.TAG_DATA, 2 * k + 1), 16)
        if k == 0:
            b = np.frombuffer(bytes([0x80]) + bytes(15), np.uint8)      # the element 1
        if not np.array_equal(o.gcm_mul(a, b), gcm_mul_int(a, b)):
            fails.append("GF(2^128) product")
            break
    if not openssl_cli.available():
        return fails + ["openssl executable not available"]
    for bits in (128, 256):
        for kk in range(nkeys):
            key = seedgen.key(92, 10 * bits + kk, bits)
            w, nr = o.expand_key(key)
            H = openssl_cli.enc("ecb", key, np.zeros(16, np.uint8))
            for ivlen, alen in ((12, 0), (12, 16), (12, 45), (1, 7), (17, 64), (60, 1000)):
                iv = seedgen.bytes_np(seedgen.stream_seed(93, seedgen.TAG_NONCE, 100 * ivlen + kk), ivlen)
                aad = seedgen.bytes_np(seedgen.stream_seed(93, seedgen.TAG_DATA, alen + kk), alen)
                _, tag = o.gcm_encrypt(w, nr, iv, aad, b"")
                if not np.array_equal(tag, openssl_cli.gmac(key, iv, aad)):
                    fails.append("GCM-%d tag of empty plaintext, IV %d B, AAD %d B" % (bits, ivlen, alen))
            for ivlen in (12, 13):
                iv = seedgen.bytes_np(seedgen.stream_seed(94, seedgen.TAG_NONCE, 100 * ivlen + kk), ivlen)
                ek_j0 = openssl_cli.gmac(key, iv, b"")
                j0 = openssl_cli.enc("ecb", key, ek_j0, decrypt=True)
                for plen, alen in ((16 * 37, 32), (1000, 0), (5, 16)):
                    pt = seedgen.data_np(95, plen + ivlen + kk, plen)
                    aad = seedgen.data_np(96, alen + kk, alen)
                    ct, tag = o.gcm_encrypt(w, nr, iv, aad, pt)
                    c0 = int.from_bytes(j0[12:].tobytes(), "big")
                    if c0 + 1 + (plen + 15) // 16 < (1 << 32):      # openssl CTR carries past 32 bits
                        icb = np.concatenate([j0[:12], np.frombuffer(((c0 + 1) & 0xFFFFFFFF).to_bytes(4, "big"),
                                                                     np.uint8)])
                        if not np.array_equal(ct, openssl_cli.enc("ctr", key, pt, iv=icb)):
                            fails.append("GCM-%d ciphertext, IV %d B" % (bits, ivlen))
                    cpad = np.concatenate([ct, np.zeros((-plen) % 16, np.uint8)])
                    g = openssl_cli.gmac(key, iv, np.concatenate([aad, cpad]))
                    l1 = np.frombuffer(_be64(8 * alen) + _be64(8 * plen), np.uint8)
                    l2 = np.frombuffer(_be64(8 * (alen + cpad.size)) + _be64(0), np.uint8)
                    if not np.array_equal(tag, g ^ gcm_mul_int(l1 ^ l2, H)):
                        fails.append("GCM-%d tag, IV %d B, %d B plaintext" % (bits, ivlen, plen))
                    back, ok = o.gcm_decrypt(w, nr, iv, aad, ct, tag)
                    if not ok or not np.array_equal(back, pt):
                        fails.append("GCM-%d decrypt" % bits)
                    if not o.gcm_decrypt(w, nr, iv, aad, ct, tag[:12])[1]:
                        fails.append("GCM-%d truncated tag rejected" % bits)
                    bad = ct.copy()
                    bad[-1] ^= 1
                    if o.gcm_decrypt(w, nr, iv, aad, bad, tag)[1]:
                        fails.append("GCM-%d changed ciphertext accepted" % bits)
                    badtag = tag.copy()
                    badtag[3] ^= 0x40
                    if o.gcm_decrypt(w, nr, iv, aad, ct, badtag)[1]:
                        fails.append("GCM-%d changed tag accepted" % bits)
                    if alen:
                        bada = aad.copy()
                        bada[0] ^= 0x80
                        if o.gcm_decrypt(w, nr, iv, bada, ct, tag)[1]:
                            fails.append("GCM-%d changed additional data accepted" % bits)
    return fails


ALL_PINS = (pin_gf, pin_sbox, pin_mix_columns, pin_shift_rows, pin_key_expansion,
            pin_openssl, pin_ctr_structure, pin_roundtrip, pin_chunking, pin_cbc, pin_xts, pin_xts_evp, pin_gcm,
            pin_gcm_evp)


def run_all(o, fast=False):
    out = {}
    for pin in ALL_PINS:
        if fast and pin is pin_gf:
            continue
        out[pin.__name__] = pin(o)
    return out
