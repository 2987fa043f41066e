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
 * run on ties (which keeps equal keys in input order).
 */
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

static void orc_msort(uint64_t *idx, uint64_t *tmp, const uint64_t *ok,
                      uint64_t lo, uint64_t hi) {
  if (hi - lo < 2) return;
  uint64_t mid = lo + (hi - lo) / 2;
  orc_msort(idx, tmp, ok, lo, mid);
  orc_msort(idx, tmp, ok, mid, hi);
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
