// Host-side arithmetic of the library: the S-box and the round tables, the
// key schedule, and the decryption schedule of the equivalent inverse cipher.
//
// GF(2^8) (FIPS-197 section 4.2) is handled here through discrete
// logarithms: {03} generates the multiplicative group of the field, so
// a*b = 3^(log a + log b) and a^-1 = 3^(255 - log a).  The S-box is the
// multiplicative inverse followed by the affine map of FIPS-197 section
// 5.1.1, written as b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ 0x63.
#include "internal.h"

#include <cstring>

namespace aesgpu {
namespace {

struct Field {
    uint8_t exp[512];
    uint8_t log[256];
    Field() {
        uint8_t x = 1;
        for (int i = 0; i < 255; i++) {
            exp[i] = x;
            log[x] = (uint8_t)i;
            // x * {03} = x * {02} + x, with x * {02} reduced by m(x)
            uint8_t x2 = (uint8_t)((x << 1) ^ ((x & 0x80) ? 0x1b : 0));
            x = (uint8_t)(x2 ^ x);
        }
        for (int i = 255; i < 512; i++)
            exp[i] = exp[i - 255];
        log[0] = 0;  // never used: products with 0 are handled apart
    }
    uint8_t mul(uint8_t a, uint8_t b) const {
        if (a == 0 || b == 0) return 0;
        return exp[log[a] + log[b]];
    }
    uint8_t inv(uint8_t a) const { return a ? exp[255 - log[a]] : 0; }
};

inline uint8_t rotl8(uint8_t b, int n) { return (uint8_t)((b << n) | (b >> (8 - n))); }

inline uint32_t pack(uint8_t b0, uint8_t b1, uint8_t b2, uint8_t b3) {
    return (uint32_t)b0 | ((uint32_t)b1 << 8) | ((uint32_t)b2 << 16) | ((uint32_t)b3 << 24);
}

inline uint32_t rotl32(uint32_t x, int n) { return n ? (x << n) | (x >> (32 - n)) : x; }

}  // namespace

const HostTables &host_tables() {
    static const HostTables t = [] {
        HostTables h;
        Field f;
        for (int x = 0; x < 256; x++) {
            uint8_t i = f.inv((uint8_t)x);
            h.sbox[x] = (uint8_t)(i ^ rotl8(i, 1) ^ rotl8(i, 2) ^ rotl8(i, 3) ^ rotl8(i, 4) ^ 0x63);
        }
        for (int x = 0; x < 256; x++)
            h.inv_sbox[h.sbox[x]] = (uint8_t)x;
        // A state column is a little-endian 32-bit word: row r in byte r.
        // te0[x] is MixColumns applied to the column (S[x], 0, 0, 0), i.e.
        // the contribution of a row-0 byte x after SubBytes; rows 1..3 are
        // the same word rotated left by 8, 16, 24 bits.  td0 is the same for
        // InvSubBytes followed by InvMixColumns (FIPS-197 section 5.3.5).
        for (int x = 0; x < 256; x++) {
            uint8_t s = h.sbox[x], is = h.inv_sbox[x];
            h.te0[x] = pack(f.mul(2, s), s, s, f.mul(3, s));
            h.td0[x] = pack(f.mul(0x0e, is), f.mul(0x09, is), f.mul(0x0d, is), f.mul(0x0b, is));
            h.isw[x] = 0x01010101u * is;
        }
        return h;
    }();
    return t;
}

int expand_key_host(const uint8_t *key, int keybits, uint32_t *w) {
    int nk;
    switch (keybits) {
    case 128: nk = 4; break;
    case 192: nk = 6; break;
    case 256: nk = 8; break;
    default: return -1;
    }
    const int nr = nk + 6;
    const HostTables &t = host_tables();
    auto sub_word = [&](uint32_t v) {
        return pack(t.sbox[v & 0xff], t.sbox[(v >> 8) & 0xff], t.sbox[(v >> 16) & 0xff],
                    t.sbox[v >> 24]);
    };
    for (int i = 0; i < nk; i++)
        w[i] = pack(key[4 * i], key[4 * i + 1], key[4 * i + 2], key[4 * i + 3]);
    uint8_t rcon = 1;
    for (int i = nk; i < 4 * (nr + 1); i++) {
        uint32_t tmp = w[i - 1];
        if (i % nk == 0) {
            // RotWord moves byte 1 to byte 0: in a little-endian word that is
            // a right rotation by 8 bits.
            tmp = sub_word(rotl32(tmp, 24)) ^ rcon;
            rcon = (uint8_t)((rcon << 1) ^ ((rcon & 0x80) ? 0x1b : 0));
        } else if (nk > 6 && i % nk == 4) {
            tmp = sub_word(tmp);
        }
        w[i] = w[i - nk] ^ tmp;
    }
    return nr;
}

uint32_t inv_mix_column_word(uint32_t col) {
    static const Field f;
    uint8_t a[4] = {(uint8_t)col, (uint8_t)(col >> 8), (uint8_t)(col >> 16), (uint8_t)(col >> 24)};
    uint8_t o[4];
    static const uint8_t m[4] = {0x0e, 0x0b, 0x0d, 0x09};
    for (int r = 0; r < 4; r++) {
        uint8_t v = 0;
        for (int c = 0; c < 4; c++)
            v ^= f.mul(m[(c - r + 4) % 4], a[c]);
        o[r] = v;
    }
    return pack(o[0], o[1], o[2], o[3]);
}

void decryption_schedule(const uint32_t *w, int nr, uint32_t *dk) {
    // Equivalent inverse cipher (FIPS-197 section 5.3.5): the round keys in
    // reverse order, with InvMixColumns applied to those of rounds 1..Nr-1.
    for (int c = 0; c < 4; c++) {
        dk[c] = w[4 * nr + c];
        dk[4 * nr + c] = w[c];
    }
    for (int r = 1; r < nr; r++)
        for (int c = 0; c < 4; c++)
            dk[4 * r + c] = inv_mix_column_word(w[4 * (nr - r) + c]);
}

}  // namespace aesgpu
