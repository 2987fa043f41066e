/*
 * Oracle: plain, slow, obviously correct CPU sort.  TEST INFRASTRUCTURE ONLY.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * link or call this.  It shares no code, header or table with the GPU library.
 *
 * What it computes (problem statement, Section 1; tie-breaking, Section 2
 * "Preliminaries" and Appendix D): given keys K[0..n) and an optional payload
 * V, output the unique permutation pi such that the pairs
 * (ord(K[pi(i)]), pi(i)) strictly increase in i, i.e. the keys in sorted order
 * with equal keys kept in input order (the position breaks ties).  The result
 * is K'[i] = K[pi(i)] bit for bit and V'[i] = V[pi(i)].
 *
 * ord: identity for uint32/uint64.  For float32 (not covered by the paper,
 * which sorts 64-bit integers) the IEEE 754-2008 totalOrder on bit patterns:
 * sign bit clear -> set the sign bit; sign bit set -> invert all bits.
 *
 * Method: textbook top-down mergesort of an index array, taking from the left
 * run on ties (which keeps equal keys in input order).  A plain parallel form
 * (oracle_sort_perm_parallel) sorts one contiguous chunk per thread with the
 * same mergesort and then merges neighbouring runs pairwise, one thread per
 * pair, round after round; the left run still wins ties, so its result is the
 * same unique permutation.  It exists to time the oracle on all host cores.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_U32 = 1, ORC_U64 = 2, ORC_F32 = 3 };

static uint64_t orc_ord(int type, const void *keys, uint64_t i) {
  if (type == ORC_U32) return ((const uint32_t *)keys)[i];
  if (type == ORC_U64) return ((const uint64_t *)keys)[i];
  uint32_t u;
  memcpy(&u, (const char *)keys + 4 * i, 4);
  if (u & 0x80000000u) return (uint32_t)~u;
  return u | 0x80000000u;
}

/* Merge the sorted runs idx[lo..mid) and idx[mid..hi) through tmp. */
static void orc_merge(uint64_t *idx, uint64_t *tmp, const uint64_t *ok,
                      uint64_t lo, uint64_t mid, uint64_t hi) {
  uint64_t i = lo, j = mid, k = lo;
  while (i < mid && j < hi) {
    /* strictly smaller right element goes first; on ties take the left one */
    if (ok[idx[j]] < ok[idx[i]])
      tmp[k++] = idx[j++];
    else
      tmp[k++] = idx[i++];
  }
  while (i < mid) tmp[k++] = idx[i++];
  while (j < hi) tmp[k++] = idx[j++];
  memcpy(idx + lo, tmp + lo, (hi - lo) * sizeof(uint64_t));
}

static void orc_msort(uint64_t *idx, uint64_t *tmp, const uint64_t *ok,
                      uint64_t lo, uint64_t hi) {
  if (hi - lo < 2) return;
  uint64_t mid = lo + (hi - lo) / 2;
  orc_msort(idx, tmp, ok, lo, mid);
  orc_msort(idx, tmp, ok, mid, hi);
  orc_merge(idx, tmp, ok, lo, mid, hi);
}

/* perm_out[i] = pi(i).  Returns 0 on success, -1 on bad type / no memory. */
int oracle_sort_perm(int type, const void *keys, uint64_t n, uint64_t *perm_out) {
  if (type != ORC_U32 && type != ORC_U64 && type != ORC_F32) return -1;
  if (n == 0) return 0;
  uint64_t *ok = (uint64_t *)malloc(n * sizeof(uint64_t));
  uint64_t *tmp = (uint64_t *)malloc(n * sizeof(uint64_t));
  if (!ok || !tmp) {
    free(ok);
    free(tmp);
    return -1;
  }
  for (uint64_t i = 0; i < n; ++i) {
    ok[i] = orc_ord(type, keys, i);
    perm_out[i] = i;
  }
  orc_msort(perm_out, tmp, ok, 0, n);
  free(ok);
  free(tmp);
  return 0;
}

/* ---- plain parallel form: chunks per thread, then a pairwise merge tree ---- */
typedef struct {
  uint64_t *idx, *tmp;
  const uint64_t *ok;
  uint64_t lo, mid, hi; /* mid == hi: sort [lo, hi); else merge the two runs */
} orc_job;

static void *orc_job_run(void *arg) {
  orc_job *j = (orc_job *)arg;
  if (j->mid == j->hi)
    orc_msort(j->idx, j->tmp, j->ok, j->lo, j->hi);
  else
    orc_merge(j->idx, j->tmp, j->ok, j->lo, j->mid, j->hi);
  return NULL;
}

/* Run the jobs on one thread each (the caller's thread takes the first). */
static int orc_run_jobs(orc_job *jobs, int nj) {
  pthread_t th[256];
  int started = 0, rc = 0;
  for (int t = 1; t < nj; ++t) {
    if (pthread_create(&th[t], NULL, orc_job_run, &jobs[t]) != 0) {
      rc = -1;
      break;
    }
    started = t;
  }
  if (nj > 0) orc_job_run(&jobs[0]);
  for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
  if (rc) /* finish what did not get a thread, on this one */
    for (int t = started + 1; t < nj; ++t) orc_job_run(&jobs[t]);
  return 0;
}

/* Same result as oracle_sort_perm, computed on `threads` threads (1..256). */
int oracle_sort_perm_parallel(int type, const void *keys, uint64_t n, uint64_t *perm_out,
                              int threads) {
  if (type != ORC_U32 && type != ORC_U64 && type != ORC_F32) return -1;
  if (threads < 1 || threads > 256) return -1;
  if (n == 0) return 0;
  if ((uint64_t)threads > n) threads = (int)n;
  uint64_t *ok = (uint64_t *)malloc(n * sizeof(uint64_t));
  uint64_t *tmp = (uint64_t *)malloc(n * sizeof(uint64_t));
  uint64_t *bound = (uint64_t *)malloc((threads + 1) * sizeof(uint64_t));
  orc_job *jobs = (orc_job *)malloc(threads * sizeof(orc_job));
  if (!ok || !tmp || !bound || !jobs) {
    free(ok);
    free(tmp);
    free(bound);
    free(jobs);
    return -1;
  }
  for (uint64_t i = 0; i < n; ++i) {
    ok[i] = orc_ord(type, keys, i);
    perm_out[i] = i;
  }
  /* run t covers [bound[t], bound[t+1]) */
  for (int t = 0; t <= threads; ++t) bound[t] = n * (uint64_t)t / (uint64_t)threads;
  for (int t = 0; t < threads; ++t) {
    orc_job j = {perm_out, tmp, ok, bound[t], bound[t + 1], bound[t + 1]};
    jobs[t] = j;
  }
  orc_run_jobs(jobs, threads);
  /* merge neighbouring runs until one is left; an odd last run waits */
  int runs = threads;
  while (runs > 1) {
    int nj = 0;
    for (int t = 0; t + 1 < runs; t += 2) {
      orc_job j = {perm_out, tmp, ok, bound[t], bound[t + 1], bound[t + 2]};
      jobs[nj++] = j;
    }
    orc_run_jobs(jobs, nj);
    int nr = 0;
    for (int t = 0; t < runs; t += 2) bound[nr++] = bound[t];
    bound[nr] = n;
    runs = nr;
  }
  free(ok);
  free(tmp);
  free(bound);
  free(jobs);
  return 0;
}

/* Sorted keys (and payload when vals != NULL) into out_keys / out_vals. */
int oracle_sort(int type, const void *keys, const uint32_t *vals, uint64_t n,
                void *out_keys, uint32_t *out_vals) {
  if (n == 0) return 0;
  uint64_t *perm = (uint64_t *)malloc(n * sizeof(uint64_t));
  if (!perm) return -1;
  int rc = oracle_sort_perm(type, keys, n, perm);
  if (rc) {
    free(perm);
    return rc;
  }
  size_t w = (type == ORC_U64) ? 8 : 4;
  for (uint64_t i = 0; i < n; ++i) {
    memcpy((char *)out_keys + w * i, (const char *)keys + w * perm[i], w);
    if (vals && out_vals) out_vals[i] = vals[perm[i]];
  }
  free(perm);
  return 0;
}
