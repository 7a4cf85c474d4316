/*
 * Oracle: a plain, slow, byte-oriented CPU implementation of AES (FIPS-197)
 * in ECB and CTR mode, and in the modes after the paper's: CBC, XTS and GCM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file.  Its users are the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg.  It shares no code, table or constant
 * generator with the GPU library: every table here is derived at start-up
 * from the GF(2^8) definitions below.
 *
 * What it computes, and where the definitions come from:
 *   - The paper (Barnes, Fernando, Mettananda, Ragel, "Improving the
 *     Throughput of the AES Algorithm with Multicore Processors",
 *     Section III-A) lists the steps: Key Expansion; an initial round that
 *     adds the round key; rounds of SubBytes, ShiftRows, MixColumns and
 *     AddRoundKey; and a final round without MixColumns.  It prints no
 *     arithmetic and no worked example, so the arithmetic of each step is
 *     written out from the AES standard (FIPS-197 sections 4, 5.1, 5.2, 5.3).
 *   - The paper never describes decryption; it is the standard's inverse
 *     cipher written in its direct form (FIPS-197 section 5.3), not the
 *     equivalent form, so that agreement with the GPU path (which uses the
 *     equivalent form) is itself a check.
 *   - Modes: the paper encrypts independent chunks and concatenates them
 *     (Section IV), which is ECB; CTR follows NIST SP 800-38A section 6.5
 *     with a 96-bit nonce and a 32-bit big-endian block counter that wraps
 *     modulo 2^32 without carrying into the nonce.  CBC is SP 800-38A
 *     section 6.2, XTS is IEEE 1619 (SP 800-38E) without ciphertext
 *     stealing, GCM is SP 800-38D sections 6 and 7.
 *
 * Style: every step is a separate function on a 4x4 byte state s[r][c]
 * (row r, column c), exactly as the standard draws it.  No T-tables, no word
 * packing, no fusion of steps.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <pthread.h>

/* ---------------------------------------------------------------------- */
/* GF(2^8) with the reduction polynomial m(x) = x^8 + x^4 + x^3 + x + 1    */
/* (FIPS-197 section 4.2).                                                 */
/* ---------------------------------------------------------------------- */

/* Multiplication by x (FIPS-197 section 4.2.1): shift left, and reduce by
 * m(x) when the bit shifted out was set. */
uint8_t ref_xtime(uint8_t b)
{
    uint8_t shifted = (uint8_t)(b << 1);
#ifdef REF_PLANT_XTIME
    return shifted;               /* planted mistake: reduction dropped */
#else
    return (b & 0x80) ? (uint8_t)(shifted ^ 0x1b) : shifted;
#endif
}

/* General multiplication by repeated xtime and addition (XOR), one bit of
 * b at a time (FIPS-197 section 4.2.1). */
uint8_t ref_gf_mul(uint8_t a, uint8_t b)
{
    uint8_t product = 0;
    while (b) {
        if (b & 1)
            product ^= a;
        a = ref_xtime(a);
        b >>= 1;
    }
    return product;
}

/* Multiplicative inverse by exhaustive search; 0 maps to 0 (FIPS-197
 * section 5.1.1). */
static uint8_t gf_inverse(uint8_t a)
{
    if (a == 0)
        return 0;
    for (int y = 1; y < 256; y++)
        if (ref_gf_mul(a, (uint8_t)y) == 1)
            return (uint8_t)y;
    return 0; /* unreachable: every non-zero element has an inverse */
}

/* The affine transformation of the S-box, bit by bit: bit i of the result
 * is b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i (indices mod 8) with
 * c = 0x63 (FIPS-197 section 5.1.1). */
static uint8_t sbox_affine(uint8_t b)
{
#ifdef REF_PLANT_AFFINE
    const uint8_t c = 0x36;       /* planted mistake: wrong constant */
#else
    const uint8_t c = 0x63;
#endif
    uint8_t out = 0;
    for (int i = 0; i < 8; i++) {
        int bit = ((b >> i) & 1)
                ^ ((b >> ((i + 4) % 8)) & 1)
                ^ ((b >> ((i + 5) % 8)) & 1)
                ^ ((b >> ((i + 6) % 8)) & 1)
                ^ ((b >> ((i + 7) % 8)) & 1)
                ^ ((c >> i) & 1);
        out |= (uint8_t)(bit << i);
    }
    return out;
}

static uint8_t SBOX[256];
static uint8_t INV_SBOX[256];
static uint8_t RCON[15];        /* RCON[j] = x^(j-1) in GF(2^8), j >= 1 */
static pthread_once_t tables_once = PTHREAD_ONCE_INIT;

static void build_tables(void)
{
    for (int x = 0; x < 256; x++)
        SBOX[x] = sbox_affine(gf_inverse((uint8_t)x));
    for (int x = 0; x < 256; x++)
        INV_SBOX[SBOX[x]] = (uint8_t)x;
    RCON[0] = 0;
    RCON[1] = 0x01;
    for (int j = 2; j < 15; j++)
        RCON[j] = ref_xtime(RCON[j - 1]);
}

static void ensure_tables(void)
{
    pthread_once(&tables_once, build_tables);
}

void ref_sbox(uint8_t out[256])
{
    ensure_tables();
    memcpy(out, SBOX, 256);
}

void ref_inv_sbox(uint8_t out[256])
{
    ensure_tables();
    memcpy(out, INV_SBOX, 256);
}

uint8_t ref_rcon(int j)
{
    ensure_tables();
    return (j >= 1 && j < 15) ? RCON[j] : 0;
}

/* ---------------------------------------------------------------------- */
/* The state: s[r][c], loaded column by column from the 16 input bytes    */
/* (FIPS-197 section 3.4: s[r][c] = in[r + 4c]).                           */
/* ---------------------------------------------------------------------- */

typedef uint8_t state_t[4][4];

static void load_state(state_t s, const uint8_t in[16])
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] = in[r + 4 * c];
}

static void store_state(uint8_t out[16], state_t s)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            out[r + 4 * c] = s[r][c];
}

/* SubBytes: every byte through the S-box (FIPS-197 section 5.1.1). */
static void sub_bytes(state_t s)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = SBOX[s[r][c]];
}

static void inv_sub_bytes(state_t s)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = INV_SBOX[s[r][c]];
}

/* ShiftRows: row r is rotated left by r positions, so the new s[r][c] is the
 * old s[r][(c + r) mod 4] (FIPS-197 section 5.1.2). */
static void shift_rows(state_t s)
{
    for (int r = 1; r < 4; r++) {
        uint8_t row[4];
        for (int c = 0; c < 4; c++)
#ifdef REF_PLANT_SHIFTROWS
            row[c] = s[r][(c + 4 - r) % 4];   /* planted mistake: wrong way */
#else
            row[c] = s[r][(c + r) % 4];
#endif
        for (int c = 0; c < 4; c++)
            s[r][c] = row[c];
    }
}

/* InvShiftRows: row r is rotated right by r positions, so the new
 * s[r][(c + r) mod 4] is the old s[r][c] (FIPS-197 section 5.3.1). */
static void inv_shift_rows(state_t s)
{
    for (int r = 1; r < 4; r++) {
        uint8_t row[4];
        for (int c = 0; c < 4; c++)
            row[(c + r) % 4] = s[r][c];
        for (int c = 0; c < 4; c++)
            s[r][c] = row[c];
    }
}

/* MixColumns on one column: multiplication by the fixed polynomial
 * {03}x^3 + {01}x^2 + {01}x + {02} modulo x^4 + 1, written as the matrix
 * product of FIPS-197 section 5.1.3. */
static void mix_column(uint8_t col[4])
{
    uint8_t a0 = col[0], a1 = col[1], a2 = col[2], a3 = col[3];
#ifdef REF_PLANT_MIXCOL
    const uint8_t three = 0x01;   /* planted mistake: {03} read as {01} */
#else
    const uint8_t three = 0x03;
#endif
    col[0] = ref_gf_mul(0x02, a0) ^ ref_gf_mul(three, a1) ^ a2 ^ a3;
    col[1] = a0 ^ ref_gf_mul(0x02, a1) ^ ref_gf_mul(three, a2) ^ a3;
    col[2] = a0 ^ a1 ^ ref_gf_mul(0x02, a2) ^ ref_gf_mul(three, a3);
    col[3] = ref_gf_mul(three, a0) ^ a1 ^ a2 ^ ref_gf_mul(0x02, a3);
}

/* InvMixColumns on one column: the inverse polynomial
 * {0b}x^3 + {0d}x^2 + {09}x + {0e} (FIPS-197 section 5.3.3). */
static void inv_mix_column(uint8_t col[4])
{
    uint8_t a0 = col[0], a1 = col[1], a2 = col[2], a3 = col[3];
    col[0] = ref_gf_mul(0x0e, a0) ^ ref_gf_mul(0x0b, a1) ^ ref_gf_mul(0x0d, a2) ^ ref_gf_mul(0x09, a3);
    col[1] = ref_gf_mul(0x09, a0) ^ ref_gf_mul(0x0e, a1) ^ ref_gf_mul(0x0b, a2) ^ ref_gf_mul(0x0d, a3);
    col[2] = ref_gf_mul(0x0d, a0) ^ ref_gf_mul(0x09, a1) ^ ref_gf_mul(0x0e, a2) ^ ref_gf_mul(0x0b, a3);
    col[3] = ref_gf_mul(0x0b, a0) ^ ref_gf_mul(0x0d, a1) ^ ref_gf_mul(0x09, a2) ^ ref_gf_mul(0x0e, a3);
}

static void mix_columns(state_t s)
{
    for (int c = 0; c < 4; c++) {
        uint8_t col[4] = { s[0][c], s[1][c], s[2][c], s[3][c] };
        mix_column(col);
        for (int r = 0; r < 4; r++)
            s[r][c] = col[r];
    }
}

static void inv_mix_columns(state_t s)
{
    for (int c = 0; c < 4; c++) {
        uint8_t col[4] = { s[0][c], s[1][c], s[2][c], s[3][c] };
        inv_mix_column(col);
        for (int r = 0; r < 4; r++)
            s[r][c] = col[r];
    }
}

/* AddRoundKey: column c of the state is XORed with word w[4*round + c];
 * byte r of that word goes into row r (FIPS-197 section 5.1.4).  The key
 * schedule is kept as 4 bytes per word, in the standard's byte order. */
static void add_round_key(state_t s, const uint8_t *w, int round)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] ^= w[(4 * round + c) * 4 + r];
}

/* Exposed single steps on a 16-byte block in the standard's column order,
 * for unit tests of the individual transformations. */
void ref_step_sub_bytes(uint8_t b[16])      { state_t s; ensure_tables(); load_state(s, b); sub_bytes(s);       store_state(b, s); }
void ref_step_inv_sub_bytes(uint8_t b[16])  { state_t s; ensure_tables(); load_state(s, b); inv_sub_bytes(s);   store_state(b, s); }
void ref_step_shift_rows(uint8_t b[16])     { state_t s; load_state(s, b); shift_rows(s);      store_state(b, s); }
void ref_step_inv_shift_rows(uint8_t b[16]) { state_t s; load_state(s, b); inv_shift_rows(s);  store_state(b, s); }
void ref_step_mix_columns(uint8_t b[16])    { state_t s; load_state(s, b); mix_columns(s);     store_state(b, s); }
void ref_step_inv_mix_columns(uint8_t b[16]){ state_t s; load_state(s, b); inv_mix_columns(s); store_state(b, s); }

/* ---------------------------------------------------------------------- */
/* KeyExpansion (FIPS-197 section 5.2; the paper's first step).            */
/* ---------------------------------------------------------------------- */

/* Expands a 128-, 192- or 256-bit key into 4*(Nr+1) words, written to w as
 * 16*(Nr+1) bytes (word i occupies bytes 4i..4i+3 in the standard's order).
 * Returns Nr (10, 12 or 14), or -1 for an unsupported key size. */
int ref_expand_key(const uint8_t *key, int keybits, uint8_t *w)
{
    int Nk, Nr;
    switch (keybits) {
    case 128: Nk = 4; Nr = 10; break;
    case 192: Nk = 6; Nr = 12; break;
    case 256: Nk = 8; Nr = 14; break;
    default:  return -1;
    }
    ensure_tables();
    for (int i = 0; i < Nk; i++)
        for (int b = 0; b < 4; b++)
            w[4 * i + b] = key[4 * i + b];

    for (int i = Nk; i < 4 * (Nr + 1); i++) {
        uint8_t temp[4];
        for (int b = 0; b < 4; b++)
            temp[b] = w[4 * (i - 1) + b];
        if (i % Nk == 0) {
            /* RotWord: cyclic left shift of the word's bytes */
            uint8_t t0 = temp[0];
            temp[0] = temp[1]; temp[1] = temp[2]; temp[2] = temp[3]; temp[3] = t0;
            /* SubWord */
            for (int b = 0; b < 4; b++)
                temp[b] = SBOX[temp[b]];
            /* Rcon[i/Nk] = (x^(i/Nk - 1), 0, 0, 0) */
#ifndef REF_PLANT_RCON
            temp[0] ^= RCON[i / Nk];
#endif
        } else if (Nk > 6 && i % Nk == 4) {
            for (int b = 0; b < 4; b++)
                temp[b] = SBOX[temp[b]];
        }
        for (int b = 0; b < 4; b++)
            w[4 * i + b] = w[4 * (i - Nk) + b] ^ temp[b];
    }
    return Nr;
}

/* ---------------------------------------------------------------------- */
/* Cipher and inverse cipher on one block.                                */
/* ---------------------------------------------------------------------- */

/* Cipher (FIPS-197 section 5.1; the paper's Section III-A step list):
 * initial AddRoundKey, Nr-1 full rounds, and a final round without
 * MixColumns. */
void ref_encrypt_block(const uint8_t *w, int Nr, const uint8_t in[16], uint8_t out[16])
{
    state_t s;
    ensure_tables();
    load_state(s, in);
    add_round_key(s, w, 0);
    for (int round = 1; round < Nr; round++) {
        sub_bytes(s);
        shift_rows(s);
        mix_columns(s);
        add_round_key(s, w, round);
    }
    sub_bytes(s);
    shift_rows(s);
#ifndef REF_PLANT_LASTKEY
    add_round_key(s, w, Nr);
#endif
    store_state(out, s);
}

/* Inverse cipher, direct form (FIPS-197 section 5.3): the steps of the
 * cipher undone in reverse order, with the round keys taken last to first. */
void ref_decrypt_block(const uint8_t *w, int Nr, const uint8_t in[16], uint8_t out[16])
{
    state_t s;
    ensure_tables();
    load_state(s, in);
    add_round_key(s, w, Nr);
    for (int round = Nr - 1; round >= 1; round--) {
        inv_shift_rows(s);
        inv_sub_bytes(s);
        add_round_key(s, w, round);
        inv_mix_columns(s);
    }
    inv_shift_rows(s);
    inv_sub_bytes(s);
    add_round_key(s, w, 0);
    store_state(out, s);
}

/* ---------------------------------------------------------------------- */
/* Modes of operation.                                                    */
/* ---------------------------------------------------------------------- */

/* ECB (SP 800-38A section 6.1): each 16-byte block on its own.  nbytes must
 * be a multiple of 16; returns -1 otherwise.  dir = 0 encrypts, 1 decrypts. */
int ref_ecb(int dir, const uint8_t *w, int Nr, const uint8_t *in, uint8_t *out, size_t nbytes)
{
    if (nbytes % 16 != 0)
        return -1;
    for (size_t j = 0; j < nbytes / 16; j++) {
        if (dir == 0)
            ref_encrypt_block(w, Nr, in + 16 * j, out + 16 * j);
        else
            ref_decrypt_block(w, Nr, in + 16 * j, out + 16 * j);
    }
    return 0;
}

/* Counter block number j (SP 800-38A section 6.5 with the standard
 * incrementing function on the last 32 bits, SP 800-38D section 6.2):
 * bytes 0..11 are those of ctr0, bytes 12..15 hold (c0 + j) mod 2^32 in
 * big-endian order, where c0 is the big-endian value of ctr0[12..15]. */
void ref_ctr_block(const uint8_t ctr0[16], uint64_t j, uint8_t T[16])
{
    uint32_t c0 = ((uint32_t)ctr0[12] << 24) | ((uint32_t)ctr0[13] << 16)
                | ((uint32_t)ctr0[14] << 8) | (uint32_t)ctr0[15];
    uint32_t c = c0 + (uint32_t)j;            /* wraps modulo 2^32 */
    memcpy(T, ctr0, 12);
#ifdef REF_PLANT_CTR_LE
    T[12] = (uint8_t)c; T[13] = (uint8_t)(c >> 8); T[14] = (uint8_t)(c >> 16); T[15] = (uint8_t)(c >> 24);
#else
    T[12] = (uint8_t)(c >> 24);
    T[13] = (uint8_t)(c >> 16);
    T[14] = (uint8_t)(c >> 8);
    T[15] = (uint8_t)c;
#endif
}

/* CTR (SP 800-38A section 6.5): output block j is input block j XOR
 * Cipher(T_j).  A final partial block uses the leading bytes of its
 * keystream block.  The same call decrypts.  first_block lets a caller
 * process a sub-range of a message: byte 0 of `in` is byte 16*first_block of
 * the message. */
void ref_ctr(const uint8_t *w, int Nr, const uint8_t ctr0[16], uint64_t first_block,
             const uint8_t *in, uint8_t *out, size_t nbytes)
{
    uint8_t T[16], K[16];
    for (size_t off = 0, j = 0; off < nbytes; off += 16, j++) {
        ref_ctr_block(ctr0, first_block + j, T);
        ref_encrypt_block(w, Nr, T, K);
        size_t n = nbytes - off < 16 ? nbytes - off : 16;
        for (size_t b = 0; b < n; b++)
            out[off + b] = in[off + b] ^ K[b];
    }
}

/* CBC (SP 800-38A section 6.2).  Encryption: C_j = Cipher(P_j XOR C_{j-1}),
 * with C_{-1} = IV.  Decryption: P_j = InvCipher(C_j) XOR C_{j-1}.  nbytes
 * must be a multiple of 16 (no padding); returns -1 otherwise.  dir = 0
 * encrypts, 1 decrypts.  `in` and `out` must not overlap. */
int ref_cbc(int dir, const uint8_t *w, int Nr, const uint8_t iv[16], const uint8_t *in, uint8_t *out,
            size_t nbytes)
{
    if (nbytes % 16 != 0)
        return -1;
    uint8_t prev[16], x[16];
    memcpy(prev, iv, 16);
    for (size_t off = 0; off < nbytes; off += 16) {
        if (dir == 0) {
            for (int b = 0; b < 16; b++)
#ifdef REF_PLANT_CBC_PLAIN
                x[b] = in[off + b] ^ (off ? in[off - 16 + b] : iv[b]);  /* planted: chains plaintext */
#else
                x[b] = in[off + b] ^ prev[b];
#endif
            ref_encrypt_block(w, Nr, x, out + off);
            memcpy(prev, out + off, 16);
        } else {
            ref_decrypt_block(w, Nr, in + off, x);
            for (int b = 0; b < 16; b++)
                out[off + b] = x[b] ^ prev[b];
            memcpy(prev, in + off, 16);
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* XTS (IEEE 1619; NIST SP 800-38E) without ciphertext stealing.          */
/* ---------------------------------------------------------------------- */

/* Multiplication of a tweak by the primitive element alpha = x in
 * GF(2^128) with the reduction polynomial x^128 + x^7 + x^2 + x + 1.  The
 * 16 bytes are a little-endian 128-bit number (byte 0 holds the lowest
 * coefficients): shift left by one bit, and if a bit falls out of the top,
 * add x^7 + x^2 + x + 1 (0x87) to byte 0. */
void ref_xts_mul_alpha(uint8_t t[16])
{
    int carry = t[15] >> 7;
    for (int b = 15; b > 0; b--)
        t[b] = (uint8_t)((t[b] << 1) | (t[b - 1] >> 7));
    t[0] = (uint8_t)(t[0] << 1);
#ifndef REF_PLANT_XTS_NOREDUCE
    if (carry)
        t[0] ^= 0x87;
#else
    (void)carry;
#endif
}

/* XTS-AES over a buffer of data units of unit_bytes bytes each (the last
 * one may be shorter; every unit is whole 16-byte blocks).  Unit u has the
 * tweak value i = first_unit + u, written as a 16-byte little-endian number
 * and encrypted with key 2; block j of the unit uses T_j = Cipher_K2(i) *
 * alpha^j, and C_j = Cipher_K1(P_j XOR T_j) XOR T_j (decryption: P_j =
 * InvCipher_K1(C_j XOR T_j) XOR T_j).  w1/w2 are the two key schedules, both
 * with Nr rounds.  Returns -1 if nbytes or unit_bytes is not a multiple of
 * 16 or unit_bytes is 0. */
int ref_xts(int dir, const uint8_t *w1, const uint8_t *w2, int Nr, size_t unit_bytes, uint64_t first_unit,
            const uint8_t *in, uint8_t *out, size_t nbytes)
{
    if (nbytes % 16 != 0 || unit_bytes == 0 || unit_bytes % 16 != 0)
        return -1;
    for (size_t u0 = 0, u = 0; u0 < nbytes; u0 += unit_bytes, u++) {
        uint8_t iv[16], t[16], x[16], y[16];
        uint64_t i = first_unit + u;
        for (int b = 0; b < 16; b++)
#ifndef REF_PLANT_XTS_BE
            iv[b] = b < 8 ? (uint8_t)(i >> (8 * b)) : 0;
#else
            iv[b] = b >= 8 ? (uint8_t)(i >> (8 * (15 - b))) : 0;
#endif
        ref_encrypt_block(w2, Nr, iv, t);
        size_t end = u0 + unit_bytes < nbytes ? u0 + unit_bytes : nbytes;
        for (size_t off = u0; off < end; off += 16) {
            for (int b = 0; b < 16; b++)
                x[b] = in[off + b] ^ t[b];
            if (dir == 0)
                ref_encrypt_block(w1, Nr, x, y);
            else
                ref_decrypt_block(w1, Nr, x, y);
            for (int b = 0; b < 16; b++)
                out[off + b] = y[b] ^ t[b];
            ref_xts_mul_alpha(t);
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* GCM (NIST SP 800-38D): CTR encryption plus the GHASH authenticator.    */
/* ---------------------------------------------------------------------- */

/* Product of two blocks in GF(2^128) (SP 800-38D section 6.3, the
 * bit-serial method).  The standard's bit order: bit 0 of a block is the
 * most significant bit of byte 0 and is the coefficient of x^0.  For each
 * bit x_i of X (i = 0..127), Z gains V when x_i is set, then V is
 * multiplied by x: shifted one bit towards the end of the block, and if the
 * bit that fell off (the coefficient of x^127) was set, R = 11100001 || 0^120
 * is added. */
void ref_gcm_mul(const uint8_t X[16], const uint8_t Y[16], uint8_t Z[16])
{
    uint8_t V[16], acc[16];
    memset(acc, 0, 16);
    memcpy(V, Y, 16);
    for (int i = 0; i < 128; i++) {
        if ((X[i / 8] >> (7 - i % 8)) & 1)
            for (int b = 0; b < 16; b++)
                acc[b] ^= V[b];
        int lsb = V[15] & 1;
        for (int b = 15; b > 0; b--)
            V[b] = (uint8_t)((V[b] >> 1) | (V[b - 1] << 7));
        V[0] >>= 1;
        if (lsb)
#ifdef REF_PLANT_GCM_R
            V[15] ^= 0x87;            /* planted: XTS's constant at the wrong end */
#else
            V[0] ^= 0xe1;
#endif
    }
    memcpy(Z, acc, 16);
}

/* GHASH (SP 800-38D section 6.4) continued over nblocks 16-byte blocks:
 * Y = (Y XOR X_i) * H for each block in turn.  Y is the running value (all
 * zero at the start of a GHASH). */
void ref_ghash(const uint8_t H[16], const uint8_t *X, size_t nblocks, uint8_t Y[16])
{
    for (size_t i = 0; i < nblocks; i++) {
        uint8_t t[16];
        for (int b = 0; b < 16; b++)
            t[b] = Y[b] ^ X[16 * i + b];
        ref_gcm_mul(t, H, Y);
    }
}

/* GHASH over a byte string padded with zeros to a whole number of blocks. */
static void ghash_padded(const uint8_t H[16], const uint8_t *X, size_t n, uint8_t Y[16])
{
    ref_ghash(H, X, n / 16, Y);
    if (n % 16) {
        uint8_t last[16];
        memset(last, 0, 16);
        memcpy(last, X + n - n % 16, n % 16);
        ref_ghash(H, last, 1, Y);
    }
}

static void put_be64(uint8_t *p, uint64_t v)
{
    for (int b = 0; b < 8; b++)
        p[b] = (uint8_t)(v >> (56 - 8 * b));
}

/* The pre-counter block J0 (SP 800-38D section 7.1, step 2): for a 96-bit
 * IV, IV || 0^31 || 1; otherwise GHASH_H(IV || 0^(s+64) || [len(IV)]_64),
 * the IV padded with zeros to whole blocks and followed by a block holding
 * its length in bits. */
void ref_gcm_j0(const uint8_t H[16], const uint8_t *iv, size_t iv_bytes, uint8_t J0[16])
{
    if (iv_bytes == 12) {
        memcpy(J0, iv, 12);
        J0[12] = 0; J0[13] = 0; J0[14] = 0; J0[15] = 1;
        return;
    }
    uint8_t lenblk[16];
    memset(J0, 0, 16);
    ghash_padded(H, iv, iv_bytes, J0);
    memset(lenblk, 0, 16);
    put_be64(lenblk + 8, 8 * (uint64_t)iv_bytes);
    ref_ghash(H, lenblk, 1, J0);
}

/* The GCM tag before truncation: S = GHASH_H(A || 0^v || C || 0^u ||
 * [len(A)]_64 || [len(C)]_64) and T = Cipher(J0) XOR S (SP 800-38D section
 * 7.1, steps 5 and 6; lengths in bits). */
static void gcm_tag(const uint8_t *w, int Nr, const uint8_t H[16], const uint8_t J0[16],
                    const uint8_t *aad, size_t aad_bytes, const uint8_t *c, size_t nbytes, uint8_t T[16])
{
    uint8_t S[16], lenblk[16], E[16];
    memset(S, 0, 16);
    ghash_padded(H, aad, aad_bytes, S);
    ghash_padded(H, c, nbytes, S);
#ifdef REF_PLANT_GCM_LEN
    put_be64(lenblk, (uint64_t)aad_bytes);          /* planted: lengths in bytes */
    put_be64(lenblk + 8, (uint64_t)nbytes);
#else
    put_be64(lenblk, 8 * (uint64_t)aad_bytes);
    put_be64(lenblk + 8, 8 * (uint64_t)nbytes);
#endif
    ref_ghash(H, lenblk, 1, S);
    ref_encrypt_block(w, Nr, J0, E);
    for (int b = 0; b < 16; b++)
        T[b] = E[b] ^ S[b];
}

/* Authenticated encryption (SP 800-38D section 7.1): H = Cipher(0^128), J0
 * from the IV, C = GCTR(inc32(J0), P) -- CTR starting one past J0 with the
 * 32-bit increment -- and the full 16-byte tag (callers truncate).  Returns
 * -1 for an empty IV. */
int ref_gcm_encrypt(const uint8_t *w, int Nr, const uint8_t *iv, size_t iv_bytes, const uint8_t *aad,
                    size_t aad_bytes, const uint8_t *in, uint8_t *out, size_t nbytes, uint8_t tag[16])
{
    if (iv_bytes == 0)
        return -1;
    uint8_t zero[16], H[16], J0[16];
    memset(zero, 0, 16);
    ref_encrypt_block(w, Nr, zero, H);
    ref_gcm_j0(H, iv, iv_bytes, J0);
    ref_ctr(w, Nr, J0, 1, in, out, nbytes);
    gcm_tag(w, Nr, H, J0, aad, aad_bytes, out, nbytes, tag);
    return 0;
}

/* Authenticated decryption (SP 800-38D section 7.2): the tag is recomputed
 * over the ciphertext and compared with the first tag_bytes bytes of `tag`.
 * The plaintext is written either way; the return value says whether it may
 * be released: 0 = authentic, 1 = FAIL, -1 = bad arguments. */
int ref_gcm_decrypt(const uint8_t *w, int Nr, const uint8_t *iv, size_t iv_bytes, const uint8_t *aad,
                    size_t aad_bytes, const uint8_t *in, uint8_t *out, size_t nbytes, const uint8_t *tag,
                    size_t tag_bytes)
{
    if (iv_bytes == 0 || tag_bytes == 0 || tag_bytes > 16)
        return -1;
    uint8_t zero[16], H[16], J0[16], T[16];
    memset(zero, 0, 16);
    ref_encrypt_block(w, Nr, zero, H);
    ref_gcm_j0(H, iv, iv_bytes, J0);
    gcm_tag(w, Nr, H, J0, aad, aad_bytes, in, nbytes, T);
    ref_ctr(w, Nr, J0, 1, in, out, nbytes);
    int diff = 0;
    for (size_t b = 0; b < tag_bytes; b++)
        diff |= T[b] ^ tag[b];
    return diff ? 1 : 0;
}
