/*
 * CPU oracle (test infrastructure only): exact transfer-matrix evaluation of
 * Eq. 2 for lattice instances, with multiword counts that cannot overflow.
 *
 * Same sweep as oracle/tm.py: sites are added in row-major order; the table
 * holds, for every state of the last W sites (the frontier; slot of site q is
 * q mod W), the best value and the number of configurations reaching it;
 * adding a site retires the oldest frontier site with a tropical sum (min
 * form, count added on ties).  Counts are little-endian arrays of `words`
 * 64-bit words; a count never exceeds 2^(number of sites added) <= 2^n, so
 * words = n / 64 + 1 always suffices.  Parallel over frontier states
 * (OpenMP).
 *
 * Spin glass (Eq. 1, energies as integers): sg_tm(Lr, Lc, right, down, h, ...)
 *   right[p] = coupling of (p, p+1) within a row, down[p] = coupling of
 *   (p, p+Lc), h[p] = field (or NULL).  sigma = 2 s - 1.
 * MWIS on a King's subgraph of an L x L grid: ksg_tm(L, present, w, ...).
 * Both return 0 on success, -1 on allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* number of threads the parallel loops use */
int tm_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

typedef struct {
  int64_t *v;     /* [S] values (min form)          */
  uint64_t *c;    /* [S * words] counts              */
} table_t;

static int alloc_table(table_t *t, int64_t S, int words) {
  t->v = (int64_t *)malloc(sizeof(int64_t) * S);
  t->c = (uint64_t *)calloc((size_t)S * words, sizeof(uint64_t));
  return (t->v && t->c) ? 0 : -1;
}

static void free_table(table_t *t) {
  free(t->v);
  free(t->c);
}

static int is_zero(const uint64_t *a, int words) {
  for (int i = 0; i < words; ++i)
    if (a[i]) return 0;
  return 1;
}

static void add_to(uint64_t *dst, const uint64_t *a, int words) {
  unsigned __int128 carry = 0;
  for (int i = 0; i < words; ++i) {
    unsigned __int128 s = (unsigned __int128)dst[i] + a[i] + carry;
    dst[i] = (uint64_t)s;
    carry = s >> 64;
  }
}

/* dst = tropical sum over the two candidates (va, ca) and (vb, cb); a zero
 * count is the tropical zero */
static void oplus2(int64_t *dv, uint64_t *dc, int64_t va, const uint64_t *ca, int64_t vb,
                   const uint64_t *cb, int words) {
  const int za = is_zero(ca, words), zb = is_zero(cb, words);
  if (za && zb) {
    *dv = 0;
    memset(dc, 0, sizeof(uint64_t) * words);
  } else if (za || (!zb && vb < va)) {
    *dv = vb;
    memcpy(dc, cb, sizeof(uint64_t) * words);
  } else if (zb || va < vb) {
    *dv = va;
    memcpy(dc, ca, sizeof(uint64_t) * words);
  } else {
    *dv = va;
    memcpy(dc, ca, sizeof(uint64_t) * words);
    add_to(dc, cb, words);
  }
}

/* final tropical sum over all states */
static void finish(const table_t *t, int64_t S, int words, int64_t *best, uint64_t *count) {
  int have = 0;
  memset(count, 0, sizeof(uint64_t) * words);
  for (int64_t s = 0; s < S; ++s) {
    const uint64_t *c = t->c + (size_t)s * words;
    if (is_zero(c, words)) continue;
    if (!have || t->v[s] < *best) {
      *best = t->v[s];
      memcpy(count, c, sizeof(uint64_t) * words);
      have = 1;
    } else if (t->v[s] == *best) {
      add_to(count, c, words);
    }
  }
}

int sg_tm(int Lr, int Lc, const int32_t *right, const int32_t *down, const int32_t *h,
          int64_t *e0, uint64_t *count, int words) {
  const int n = Lr * Lc, W = Lc;
  const int64_t S = (int64_t)1 << W;
  table_t cur, nxt;
  if (alloc_table(&cur, S, words) || alloc_table(&nxt, S, words)) return -1;
  for (int64_t s = 0; s < S; ++s) cur.v[s] = 0;
  cur.c[0] = 1; /* sites not yet added sit in state 0 */
  for (int p = 0; p < n; ++p) {
    const int r = p / Lc, col = p % Lc, b = p % W;
    const int64_t hp = h ? h[p] : 0;
#pragma omp parallel for schedule(static)
    for (int64_t lo = 0; lo < S; ++lo) {
      if ((lo >> b) & 1) continue; /* enumerate states with slot b clear */
      const int64_t hi = lo | ((int64_t)1 << b);
      for (int t = 0; t < 2; ++t) { /* new spin */
        const int64_t sp = 2 * t - 1;
        int64_t base = -hp * sp;
        if (col > 0) {
          const int64_t sl = (((lo >> ((p - 1) % W)) & 1) * 2) - 1;
          base -= (int64_t)right[p - 1] * sl * sp;
        }
        int64_t cv[2];
        for (int u = 0; u < 2; ++u) { /* retired site p - W */
          const int64_t src = u ? hi : lo;
          cv[u] = cur.v[src] + base;
          if (r > 0) cv[u] -= (int64_t)down[p - W] * (2 * u - 1) * sp;
        }
        const int64_t dst = t ? hi : lo;
        oplus2(&nxt.v[dst], nxt.c + (size_t)dst * words, cv[0], cur.c + (size_t)lo * words, cv[1],
               cur.c + (size_t)hi * words, words);
      }
    }
    table_t tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  finish(&cur, S, words, e0, count);
  free_table(&cur);
  free_table(&nxt);
  return 0;
}

int ksg_tm(int L, const uint8_t *present, const int32_t *w, int64_t *wmax, uint64_t *count,
           int words) {
  const int W = L + 1, n = L * L;
  const int64_t S = (int64_t)1 << W;
  table_t cur, nxt;
  if (alloc_table(&cur, S, words) || alloc_table(&nxt, S, words)) return -1;
  for (int64_t s = 0; s < S; ++s) cur.v[s] = 0;
  cur.c[0] = 1;
  uint64_t *zero = (uint64_t *)calloc(words, sizeof(uint64_t));
  if (!zero) return -1;
  for (int p = 0; p < n; ++p) {
    const int r = p / L, col = p % L, b = p % W;
    /* occupied earlier king neighbours: left, up-left, up, up-right */
    int nb[4], nn = 0;
    if (col > 0 && present[p - 1]) nb[nn++] = p - 1;
    if (r > 0)
      for (int dc = -1; dc <= 1; ++dc) {
        const int cc = col + dc;
        if (cc >= 0 && cc < L && present[p - L + dc]) nb[nn++] = p - L + dc;
      }
#pragma omp parallel for schedule(static)
    for (int64_t lo = 0; lo < S; ++lo) {
      if ((lo >> b) & 1) continue;
      const int64_t hi = lo | ((int64_t)1 << b);
      for (int t = 0; t < 2; ++t) {
        const int64_t dst = t ? hi : lo;
        if (t == 1 && !present[p]) { /* absent site: state 1 does not exist */
          nxt.v[dst] = 0;
          memset(nxt.c + (size_t)dst * words, 0, sizeof(uint64_t) * words);
          continue;
        }
        int ok_other = 1, retired_nb = 0;
        if (t == 1)
          for (int i = 0; i < nn; ++i) {
            if (nb[i] == p - W) { retired_nb = 1; continue; }
            if ((lo >> (nb[i] % W)) & 1) ok_other = 0;
          }
        int64_t cv[2];
        const uint64_t *cc[2];
        for (int u = 0; u < 2; ++u) {
          const int64_t src = u ? hi : lo;
          cv[u] = cur.v[src] - (int64_t)w[p] * t;
          const int ok = ok_other && !(t == 1 && u == 1 && retired_nb);
          cc[u] = ok ? cur.c + (size_t)src * words : zero;
        }
        oplus2(&nxt.v[dst], nxt.c + (size_t)dst * words, cv[0], cc[0], cv[1], cc[1], words);
      }
    }
    table_t tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  int64_t best = 0;
  finish(&cur, S, words, &best, count);
  *wmax = -best;
  free(zero);
  free_table(&cur);
  free_table(&nxt);
  return 0;
}
