/*
 * Oracle, parallel runner: the paper's own multicore method (Section IV-B,
 * pthreads variant) applied to the plain oracle of aes_ref.c.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, and the benchmark's CPU
 * baseline).  The paper splits the input into as many chunks as there are
 * parallel instances (Section IV-A), creates one thread per chunk, encrypts
 * each chunk in its thread, joins the threads and then joins the outputs.
 * Here the chunks are whole 16-byte blocks (chunk k holds blocks
 * [floor(kB/T), floor((k+1)B/T)) of B blocks) and every thread writes its
 * chunk at its own offset in one output buffer, which is the same result as
 * concatenating the per-chunk outputs.  For CTR, chunk k starts its counter
 * at block floor(kB/T) of the message; a final partial block belongs to the
 * last chunk.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <time.h>
#include <pthread.h>

int  ref_ecb(int dir, const uint8_t *w, int Nr, const uint8_t *in, uint8_t *out, size_t nbytes);
void ref_ctr(const uint8_t *w, int Nr, const uint8_t ctr0[16], uint64_t first_block,
             const uint8_t *in, uint8_t *out, size_t nbytes);

enum { REF_OP_ECB_ENC = 0, REF_OP_ECB_DEC = 1, REF_OP_CTR = 2 };

typedef struct {
    int op;
    const uint8_t *w;
    int Nr;
    const uint8_t *ctr0;
    const uint8_t *in;
    uint8_t *out;
    size_t first_block;   /* first block of this chunk */
    size_t nbytes;        /* bytes of this chunk */
} chunk_job;

static void *run_chunk(void *arg)
{
    chunk_job *j = (chunk_job *)arg;
    size_t off = 16 * j->first_block;
    if (j->op == REF_OP_CTR)
        ref_ctr(j->w, j->Nr, j->ctr0, j->first_block, j->in + off, j->out + off, j->nbytes);
    else
        ref_ecb(j->op == REF_OP_ECB_DEC, j->w, j->Nr, j->in + off, j->out + off, j->nbytes);
    return NULL;
}

/* Runs `op` over nbytes of `in` into `out` with `nthreads` threads, one
 * contiguous chunk each.  Wall time from the first pthread_create to the
 * last pthread_join (CLOCK_MONOTONIC) goes to *seconds if it is not NULL.
 * Returns 0, or -1 for bad arguments (ECB length not a multiple of 16,
 * nthreads < 1) or a thread that could not be created. */
int ref_par_run(int op, const uint8_t *w, int Nr, const uint8_t *ctr0,
                const uint8_t *in, uint8_t *out, size_t nbytes, int nthreads,
                double *seconds)
{
    if (nthreads < 1 || (op != REF_OP_CTR && nbytes % 16 != 0) ||
        op < REF_OP_ECB_ENC || op > REF_OP_CTR)
        return -1;
    size_t nblocks = (nbytes + 15) / 16;
    chunk_job *jobs = (chunk_job *)calloc((size_t)nthreads, sizeof(chunk_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int *started = (int *)calloc((size_t)nthreads, sizeof(int));
    if (!jobs || !tid || !started) {
        free(jobs); free(tid); free(started);
        return -1;
    }
    for (int k = 0; k < nthreads; k++) {
        size_t b0 = (size_t)((unsigned __int128)nblocks * (unsigned)k / (unsigned)nthreads);
        size_t b1 = (size_t)((unsigned __int128)nblocks * (unsigned)(k + 1) / (unsigned)nthreads);
        size_t end = 16 * b1 < nbytes ? 16 * b1 : nbytes;
        jobs[k].op = op; jobs[k].w = w; jobs[k].Nr = Nr; jobs[k].ctr0 = ctr0;
        jobs[k].in = in; jobs[k].out = out;
        jobs[k].first_block = b0;
        jobs[k].nbytes = end > 16 * b0 ? end - 16 * b0 : 0;
    }

    int rc = 0;
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int k = 0; k < nthreads; k++) {
        if (pthread_create(&tid[k], NULL, run_chunk, &jobs[k]) != 0) {
            rc = -1;
            break;
        }
        started[k] = 1;
    }
    for (int k = 0; k < nthreads; k++)
        if (started[k])
            pthread_join(tid[k], NULL);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    if (seconds)
        *seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    free(jobs); free(tid); free(started);
    return rc;
}
