/*
 * bsp_oracle_mt.c -- TEST INFRASTRUCTURE ONLY: the CPU oracle of
 * bsp_oracle.c with its per-processor steps spread over host threads.
 *
 * The simulated BSP processors do their local work independently: each step
 * of bsp_oracle.c (local sort O2, partition O6, routing O8, merge O9) writes
 * only its own processor's share of the output arrays. This driver runs those
 * same step functions for processors q = t, t + T, t + 2T, ... on host thread
 * t of T, with a join between steps (the supersteps). The sample, the
 * splitters and the prefix sums stay sequential. The result is byte-identical
 * to ora_sort (checked by the CPU tests); it exists so that the oracle can be
 * timed on all host cores and run at the full workload sizes in tests.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_ENOMEM 2

/* From bsp_oracle.c. */
struct ora_run;
typedef void (*ora_step_fn)(struct ora_run* R, int q, void* scratch);
typedef int (*ora_each_fn)(struct ora_run* R, int count, ora_step_fn step, size_t scratch_bytes, void* ctx);
int ora_sort_driver(const uint64_t* ok, int64_t n, int p, int s, int variant, uint64_t seed,
                    int64_t* perm, int64_t* B_idx_out, uint64_t* smp_key, int64_t* smp_pos,
                    uint64_t* spl_key, int64_t* spl_pos, int64_t* C_out, int64_t* Z_idx_out,
                    int untagged, ora_each_fn each, void* ctx);

typedef struct {
    struct ora_run* R;
    int count, t, T;
    ora_step_fn step;
    size_t scratch_bytes;
    int rc;
} job_t;

static void* worker(void* arg) {
    job_t* j = (job_t*)arg;
    void* scratch = malloc(j->scratch_bytes);
    if (!scratch) { j->rc = ORA_ENOMEM; return NULL; }
    for (int q = j->t; q < j->count; q += j->T) j->step(j->R, q, scratch);
    free(scratch);
    j->rc = ORA_OK;
    return NULL;
}

static int each_threads(struct ora_run* R, int count, ora_step_fn step, size_t scratch_bytes, void* ctx) {
    int T = *(const int*)ctx;
    if (T > count) T = count;
    if (T < 1) T = 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)T);
    job_t* jobs = (job_t*)malloc(sizeof(job_t) * (size_t)T);
    if (!th || !jobs) { free(th); free(jobs); return ORA_ENOMEM; }
    int started = 0, rc = ORA_OK;
    for (int t = 0; t < T; t++) {
        jobs[t].R = R; jobs[t].count = count; jobs[t].t = t; jobs[t].T = T;
        jobs[t].step = step; jobs[t].scratch_bytes = scratch_bytes; jobs[t].rc = ORA_ENOMEM;
        if (pthread_create(&th[t], NULL, worker, &jobs[t]) != 0) {
            /* run what could not be started on this thread */
            worker(&jobs[t]);
            if (jobs[t].rc) rc = jobs[t].rc;
            jobs[t].rc = -1;
            continue;
        }
        started++;
    }
    for (int t = 0; t < T; t++) {
        if (jobs[t].rc == -1) continue;
        pthread_join(th[t], NULL);
        if (jobs[t].rc) rc = jobs[t].rc;
    }
    (void)started;
    free(th);
    free(jobs);
    return rc;
}

/* ora_sort with the per-processor steps on `threads` host threads. */
int ora_sort_mt(const uint64_t* ok, int64_t n, int p, int s, int variant, uint64_t seed,
                int64_t* perm, int64_t* B_idx_out, uint64_t* smp_key, int64_t* smp_pos,
                uint64_t* spl_key, int64_t* spl_pos, int64_t* C_out, int64_t* Z_idx_out, int threads) {
    return ora_sort_driver(ok, n, p, s, variant, seed, perm, B_idx_out, smp_key, smp_pos, spl_key, spl_pos,
                           C_out, Z_idx_out, 0, each_threads, &threads);
}
