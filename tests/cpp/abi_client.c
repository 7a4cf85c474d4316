/*
 * A plain C client of the library's C ABI (include/aesgpu.h): no Python and
 * no torch, only the HIP runtime for device memory.  It reads one job file,
 * runs ECB, CTR, XTS and GCM on the GPU through the exported calls, and writes
 * the outputs for the test to compare with the oracle.
 *
 * Job file (little-endian): key[32] key2[32] keybits:u32 unit_bytes:u32
 * first_unit:u64 ctr0[16] aad_bytes:u32 nbytes:u64 aad[aad_bytes] data[nbytes].
 * Output file: ecb[n16] ctr[nbytes] xts[n16] gcm[nbytes] tag[16] status[4]:i32,
 * where n16 = nbytes rounded down to whole blocks and status holds, in order,
 * the GCM verdict on the right tag, on a changed tag, ECB round trip equal,
 * XTS round trip equal.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "aesgpu.h"

#define CHECK_AES(call)                                                              \
    do {                                                                             \
        int st_ = (call);                                                            \
        if (st_ != AES_OK) {                                                         \
            fprintf(stderr, "%s failed: %d (%s)\n", #call, st_, aes_last_error());   \
            exit(2);                                                                 \
        }                                                                            \
    } while (0)
#define CHECK_HIP(call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));        \
            exit(3);                                                                 \
        }                                                                            \
    } while (0)

static void read_exact(FILE *f, void *p, size_t n) {
    if (n && fread(p, 1, n, f) != n) {
        fprintf(stderr, "short job file\n");
        exit(4);
    }
}

static void *dev_alloc(size_t n) {
    void *p = NULL;
    CHECK_HIP(hipMalloc(&p, n ? n : 16));
    return p;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s job.bin out.bin\n", argv[0]);
        return 1;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) {
        perror("job");
        return 1;
    }
    uint8_t key[32], key2[32], ctr0[16];
    uint32_t keybits, unit_bytes, aad_bytes;
    uint64_t first_unit, nbytes;
    read_exact(f, key, 32);
    read_exact(f, key2, 32);
    read_exact(f, &keybits, 4);
    read_exact(f, &unit_bytes, 4);
    read_exact(f, &first_unit, 8);
    read_exact(f, ctr0, 16);
    read_exact(f, &aad_bytes, 4);
    read_exact(f, &nbytes, 8);
    uint8_t *aad = malloc(aad_bytes ? aad_bytes : 1), *data = malloc(nbytes ? nbytes : 1);
    read_exact(f, aad, aad_bytes);
    read_exact(f, data, nbytes);
    fclose(f);
    const size_t n16 = nbytes & ~(size_t)15;

    uint8_t rk[240], rk2[240];
    int nr = 0, nr2 = 0;
    CHECK_AES(aes_expand_key(key, (int)keybits, rk, &nr));
    CHECK_AES(aes_expand_key(key2, (int)keybits, rk2, &nr2));

    uint8_t *d_in = dev_alloc(nbytes), *d_out = dev_alloc(nbytes), *d_back = dev_alloc(nbytes);
    uint8_t *d_aad = dev_alloc(aad_bytes), *d_tag = dev_alloc(16), *d_tag2 = dev_alloc(16);
    int *d_ok = dev_alloc(sizeof(int));
    size_t ws_bytes = 0;
    CHECK_AES(aes_gcm_workspace_size(&ws_bytes));
    void *d_ws = dev_alloc(ws_bytes);
    CHECK_HIP(hipMemcpy(d_in, data, nbytes, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_aad, aad, aad_bytes, hipMemcpyHostToDevice));

    uint8_t *ecb = malloc(n16 ? n16 : 1), *ctr = malloc(nbytes ? nbytes : 1);
    uint8_t *xts = malloc(n16 ? n16 : 1), *gcm = malloc(nbytes ? nbytes : 1), *back = malloc(nbytes ? nbytes : 1);
    uint8_t tag[16];
    int32_t status[4] = {-1, -1, -1, -1};

    /* ECB and its round trip */
    CHECK_AES(aes_encrypt(d_in, d_out, n16, rk, nr, AES_MODE_ECB, NULL, NULL));
    CHECK_AES(aes_decrypt(d_out, d_back, n16, rk, nr, AES_MODE_ECB, NULL, NULL));
    CHECK_HIP(hipMemcpy(ecb, d_out, n16, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(back, d_back, n16, hipMemcpyDeviceToHost));
    status[2] = memcmp(back, data, n16) == 0;

    /* CTR over the whole length */
    CHECK_AES(aes_encrypt(d_in, d_out, nbytes, rk, nr, AES_MODE_CTR, ctr0, NULL));
    CHECK_HIP(hipMemcpy(ctr, d_out, nbytes, hipMemcpyDeviceToHost));

    /* XTS and its round trip */
    CHECK_AES(aes_xts_encrypt(d_in, d_out, n16, rk, rk2, nr, unit_bytes, first_unit, NULL));
    CHECK_AES(aes_xts_decrypt(d_out, d_back, n16, rk, rk2, nr, unit_bytes, first_unit, NULL));
    CHECK_HIP(hipMemcpy(xts, d_out, n16, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(back, d_back, n16, hipMemcpyDeviceToHost));
    status[3] = memcmp(back, data, n16) == 0;

    /* GCM with the first 12 bytes of ctr0 as the IV; then the verdicts */
    CHECK_AES(aes_gcm_encrypt(d_in, d_out, nbytes, d_aad, aad_bytes, rk, nr, ctr0, 12, d_tag, d_ws, ws_bytes,
                              NULL));
    CHECK_HIP(hipMemcpy(gcm, d_out, nbytes, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(tag, d_tag, 16, hipMemcpyDeviceToHost));
    int ok = -1;
    CHECK_AES(aes_gcm_decrypt(d_out, d_back, nbytes, d_aad, aad_bytes, rk, nr, ctr0, 12, d_tag, 16, d_ok, d_ws,
                              ws_bytes, NULL));
    CHECK_HIP(hipMemcpy(&ok, d_ok, sizeof(int), hipMemcpyDeviceToHost));
    status[0] = ok;
    uint8_t bad[16];
    memcpy(bad, tag, 16);
    bad[0] ^= 1;
    CHECK_HIP(hipMemcpy(d_tag2, bad, 16, hipMemcpyHostToDevice));
    CHECK_AES(aes_gcm_decrypt(d_out, d_back, nbytes, d_aad, aad_bytes, rk, nr, ctr0, 12, d_tag2, 16, d_ok, d_ws,
                              ws_bytes, NULL));
    CHECK_HIP(hipMemcpy(&ok, d_ok, sizeof(int), hipMemcpyDeviceToHost));
    status[1] = ok;
    CHECK_HIP(hipDeviceSynchronize());

    FILE *o = fopen(argv[2], "wb");
    if (!o) {
        perror("out");
        return 1;
    }
    fwrite(ecb, 1, n16, o);
    fwrite(ctr, 1, nbytes, o);
    fwrite(xts, 1, n16, o);
    fwrite(gcm, 1, nbytes, o);
    fwrite(tag, 1, 16, o);
    fwrite(status, 4, 4, o);
    fclose(o);
    printf("abi client ok\n");
    return 0;
}
