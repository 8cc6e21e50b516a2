/*
 * oracle.c -- CPU oracle for least-model evaluation of the transitive-closure
 * and same-generation programs.  TEST INFRASTRUCTURE ONLY: it is called by
 * tests/, by the smoke check and by the bench's CPU-baseline leg, never by the
 * product path, and it shares no code with the GPU library.
 *
 * Everything here is plain, single-pass code on bitset rows (64 constants per
 * word), chosen to be checked by eye against the definitions it follows:
 *
 *   - The semantics is the least Herbrand model reached by iterating the
 *     immediate-consequence operator T_DB from the empty set (Sec. 2).  The
 *     oracle runs it semi-naively: a round only joins the facts that were new
 *     in the previous round.  Both programs here are linear (one recursive
 *     goal per rule body), so the facts known after round k are exactly the
 *     k-th element of the matrix series of Sec. 3 (R^(0) = 0,
 *     R^(k+1) = min1(R1 + R1 R^(k))) and of its same-generation counterpart.
 *
 *   - Transitive closure: rules r2(x,z) <- r1(x,z) and
 *     r2(x,z) <- r1(x,y), r2(y,z) (program DB1 of Sec. 3).
 *   - Same generation: r2(x,w) <- diag(x,w) and
 *     r2(x,w) <- r1(x,y), r2(y,z), r1(w,z) (Sec. 7.2, right-hand program).
 *   - Repeated squaring: the non-linear program r2 <- r2 /\ r2 of Sec. 8,
 *     whose matrix series R^(k+1) = min1(R1 + R^(k) R^(k)) is evaluated
 *     literally by or_tc_square_literal.
 *   - Brute force for cross-checks: Warshall's algorithm (the paper's own
 *     correctness pre-experiment, Sec. 7.1) and one breadth-first search per
 *     source, which also yields path-length histograms.
 *
 * Conventions: a relation over n constants is a dense uint8 n x n matrix,
 * row-major, entry (i, j) != 0 iff r(e_i, e_j) holds (row = first argument,
 * Sec. 2).  Outputs are written as exact 0/1 bytes.  ones[k] receives the
 * number of true entries of the k-th iterate, for k = 0 .. iters.
 * "iters" counts applications of the update starting from the empty relation,
 * including the first one that changes nothing.
 *
 * Return value: 0 on success, 1 if maxsteps was reached first (the result is
 * then the last iterate computed), 2 on allocation failure, 3 on bad input.
 */
#define _POSIX_C_SOURCE 200809L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef uint64_t word;

static int64_t nwords(int64_t n) { return (n + 63) / 64; }

static int64_t popcount_row(const word* r, int64_t w) {
  int64_t c = 0;
  for (int64_t i = 0; i < w; ++i) c += __builtin_popcountll(r[i]);
  return c;
}

static void set_bit(word* r, int64_t j) { r[j >> 6] |= (word)1 << (j & 63); }
static int get_bit(const word* r, int64_t j) { return (int)((r[j >> 6] >> (j & 63)) & 1); }

/* Dense uint8 -> bitset rows. */
static word* dense_to_bits(int64_t n, const uint8_t* a) {
  int64_t w = nwords(n);
  word* b = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  if (!b) return NULL;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j)
      if (a[i * n + j]) set_bit(b + i * w, j);
  return b;
}

static void bits_to_dense(int64_t n, const word* b, uint8_t* out) {
  int64_t w = nwords(n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) out[i * n + j] = (uint8_t)get_bit(b + i * w, j);
}

/* Successor lists (CSR) of a dense relation: succ(i) = { j : a[i][j] != 0 }. */
typedef struct { int64_t* ptr; int32_t* idx; } csr;

static int build_csr(int64_t n, const uint8_t* a, int transpose, csr* g) {
  g->ptr = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
  if (!g->ptr) return 2;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j)
      if (a[i * n + j]) g->ptr[(transpose ? j : i) + 1]++;
  for (int64_t i = 0; i < n; ++i) g->ptr[i + 1] += g->ptr[i];
  g->idx = (int32_t*)malloc((size_t)(g->ptr[n] + 1) * sizeof(int32_t));
  int64_t* fill = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
  if (!g->idx || !fill) { free(fill); return 2; }
  memcpy(fill, g->ptr, (size_t)n * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j)
      if (a[i * n + j]) {
        if (transpose) g->idx[fill[j]++] = (int32_t)i;
        else g->idx[fill[i]++] = (int32_t)j;
      }
  free(fill);
  return 0;
}

static void free_csr(csr* g) { free(g->ptr); free(g->idx); }

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Transitive closure, semi-naive.  Round 1 derives r2 from the exit rule:
 * T_1 = Delta_1 = r1.  Round k+1 joins r1 with the facts new in round k:
 *   Delta_{k+1}(x) = ( OR_{y in succ(x)} Delta_k(y) ) \ T_k(x),
 *   T_{k+1} = T_k  u  Delta_{k+1}.
 * Stops at the first empty Delta (that round is counted in iters) or after
 * maxsteps rounds, in which case T holds T_maxsteps.
 *
 * tc_rounds runs the rounds after round 1: on entry *T = *D = T_1 (bitset
 * rows, w words each), Dn is scratch of the same size and ones[1] holds
 * |T_1|.  *D and *Dn may be swapped on return.  Returns 0 or 1 as below and
 * leaves the number of rounds in *k.
 */
static int tc_rounds(int64_t n, int64_t w, const csr* g, word* T, word** Dp, word** Dnp, int64_t* ones,
                     int64_t maxsteps, int64_t* kp) {
  word* D = *Dp;
  word* Dn = *Dnp;
  int rc = 0;
  int64_t k = 1;
  int64_t delta = ones ? ones[1] : 1;
  if (!ones) {
    delta = 0;
    for (int64_t i = 0; i < n; ++i) delta += popcount_row(T + i * w, w);
  }
  while (delta != 0) {
    if (k == maxsteps) { rc = 1; break; }
    delta = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : delta)
    for (int64_t x = 0; x < n; ++x) {
      word* dst = Dn + x * w;
      memset(dst, 0, (size_t)w * sizeof(word));
      for (int64_t e = g->ptr[x]; e < g->ptr[x + 1]; ++e) {
        const word* src = D + (int64_t)g->idx[e] * w;
        for (int64_t q = 0; q < w; ++q) dst[q] |= src[q];
      }
      word* t = T + x * w;
      for (int64_t q = 0; q < w; ++q) { dst[q] &= ~t[q]; t[q] |= dst[q]; }
      delta += popcount_row(dst, w);
    }
    word* tmp = D; D = Dn; Dn = tmp;
    ++k;
    if (ones) ones[k] = ones[k - 1] + delta;
  }
  *Dp = D;
  *Dnp = Dn;
  *kp = k;
  return rc;
}

int or_tc_seminaive(int64_t n, const uint8_t* A, uint8_t* R, int64_t* ones, int64_t maxsteps,
                    int64_t* iters) {
  if (n < 0 || maxsteps < 0) return 3;
  int64_t w = nwords(n);
  csr g;
  if (build_csr(n, A, 0, &g)) return 2;
  word* T = dense_to_bits(n, A);
  word* D = dense_to_bits(n, A);
  word* Dn = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  if (!T || !D || !Dn) { free(T); free(D); free(Dn); free_csr(&g); return 2; }
  int rc = 0;
  int64_t k = 0;
  if (ones) ones[0] = 0;
  if (maxsteps == 0) {
    memset(T, 0, (size_t)(n * w) * sizeof(word));
  } else {
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) c += popcount_row(T + i * w, w);
    if (ones) ones[1] = c;
    rc = tc_rounds(n, w, &g, T, &D, &Dn, ones, maxsteps, &k);
  }
  if (iters) *iters = k;
  if (R) bits_to_dense(n, T, R);
  free(T); free(D); free(Dn); free_csr(&g);
  return rc;
}

/*
 * The same closure from an edge list, with the rounds timed on their own.
 * edges holds m pairs (i, j), row-major [m x 2], meaning r1(e_i, e_j);
 * pairs outside [0, n) are ignored and repeated pairs count once.  Set-up
 * (successor lists and T_1 = Delta_1 as bitset rows) is not timed; *seconds
 * receives the monotonic-clock time of the rounds alone, from T_1 in memory
 * to the model in memory.  model_ones receives |model|; R (dense n x n,
 * optional) receives the model after the clock has stopped.  threads > 0
 * sets the OpenMP thread count for the call; *threads_used reports it.
 */
int or_tc_seminaive_edges(int64_t n, int64_t m, const int32_t* edges, int threads, uint8_t* R,
                          int64_t* model_ones, int64_t* iters, double* seconds, int* threads_used) {
  if (n < 0 || m < 0 || (m > 0 && !edges)) return 3;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
  if (threads_used) *threads_used = omp_get_max_threads();
#else
  (void)threads;
  if (threads_used) *threads_used = 1;
#endif
  int64_t w = nwords(n);
  word* T = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  word* D = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  word* Dn = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  csr g = {(int64_t*)calloc((size_t)(n + 1), sizeof(int64_t)), NULL};
  if (!T || !D || !Dn || !g.ptr) { free(T); free(D); free(Dn); free(g.ptr); return 2; }
  /* distinct pairs as bitset rows, then successor lists read off the rows */
  for (int64_t e = 0; e < m; ++e) {
    int64_t i = edges[2 * e], j = edges[2 * e + 1];
    if (i >= 0 && i < n && j >= 0 && j < n) set_bit(T + i * w, j);
  }
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t ri = popcount_row(T + i * w, w);
    g.ptr[i + 1] = g.ptr[i] + ri;
    c += ri;
  }
  g.idx = (int32_t*)malloc((size_t)(c + 1) * sizeof(int32_t));
  if (!g.idx) { free(T); free(D); free(Dn); free_csr(&g); return 2; }
  for (int64_t i = 0; i < n; ++i) {
    int64_t f = g.ptr[i];
    for (int64_t j = 0; j < n; ++j)
      if (get_bit(T + i * w, j)) g.idx[f++] = (int32_t)j;
  }
  memcpy(D, T, (size_t)(n * w) * sizeof(word));
  int64_t k = 0;
  int64_t* ones = (int64_t*)calloc((size_t)(n + 3), sizeof(int64_t));
  if (!ones) { free(T); free(D); free(Dn); free_csr(&g); return 2; }
  ones[1] = c;
  struct timespec t0, t1;
  clock_gettime(CLOCK_MONOTONIC, &t0);
  int rc = n == 0 ? 0 : tc_rounds(n, w, &g, T, &D, &Dn, ones, n + 2, &k);
  clock_gettime(CLOCK_MONOTONIC, &t1);
  if (n == 0) k = 1;
  if (seconds) *seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
  if (iters) *iters = k;
  if (model_ones) *model_ones = ones[k];
  if (R) bits_to_dense(n, T, R);
  free(ones); free(T); free(D); free(Dn); free_csr(&g);
  return rc;
}

/*
 * Repeated squaring, taken literally: R^(0) = 0, R^(k+1) = min1(A + R^(k) R^(k)).
 * With Boolean rows, (R R)(i) = OR_{m in R(i)} R(m).  Jacobi order: every row
 * of the new iterate reads only the previous iterate.
 */
int or_tc_square_literal(int64_t n, const uint8_t* A, uint8_t* R, int64_t* ones, int64_t maxsteps,
                         int64_t* iters) {
  if (n < 0 || maxsteps < 0) return 3;
  int64_t w = nwords(n);
  word* Ab = dense_to_bits(n, A);
  word* Rc = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  word* Rn = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  if (!Ab || !Rc || !Rn) { free(Ab); free(Rc); free(Rn); return 2; }
  int rc = 0;
  int64_t k = 0;
  if (ones) ones[0] = 0;
  for (;;) {
    if (k == maxsteps) { rc = 1; break; }
    int64_t c = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : c)
    for (int64_t i = 0; i < n; ++i) {
      word* dst = Rn + i * w;
      const word* ri = Rc + i * w;
      memcpy(dst, Ab + i * w, (size_t)w * sizeof(word));
      for (int64_t m = 0; m < n; ++m)
        if (get_bit(ri, m)) {
          const word* rm = Rc + m * w;
          for (int64_t q = 0; q < w; ++q) dst[q] |= rm[q];
        }
      c += popcount_row(dst, w);
    }
    ++k;
    if (ones) ones[k] = c;
    int same = memcmp(Rc, Rn, (size_t)(n * w) * sizeof(word)) == 0;
    word* tmp = Rc; Rc = Rn; Rn = tmp;
    if (same) break;
  }
  if (iters) *iters = k;
  if (R) bits_to_dense(n, Rc, R);
  free(Ab); free(Rc); free(Rn);
  return rc;
}

/*
 * Warshall's algorithm on bitset rows: for each intermediate constant m, every
 * row that reaches m also reaches everything m reaches.  Starting from A it
 * yields the pairs joined by a path of length >= 1.
 */
int or_warshall(int64_t n, const uint8_t* A, uint8_t* R) {
  if (n < 0) return 3;
  int64_t w = nwords(n);
  word* B = dense_to_bits(n, A);
  if (!B) return 2;
  for (int64_t m = 0; m < n; ++m) {
    const word* bm = B + m * w;
    for (int64_t i = 0; i < n; ++i) {
      word* bi = B + i * w;
      if (get_bit(bi, m))
        for (int64_t q = 0; q < w; ++q) bi[q] |= bm[q];
    }
  }
  bits_to_dense(n, B, R);
  free(B);
  return 0;
}

/*
 * One breadth-first search per source row, over successor lists.
 * For a pair (s, t) let d+(s, t) be the length of a shortest path of length
 * >= 1 from s to t (for t != s the BFS distance; for t == s one plus the
 * smallest BFS distance from s to a predecessor of s).
 *   hist[L]  += number of pairs with d+ = L   (hist has n+2 entries)
 *   R (optional, dense n x n): R[s][t] = 1 iff d+(s,t) is defined.
 *   rows/nrows (optional): restrict the sources to the listed rows; R then
 *   has nrows rows, in that order.
 */
int or_bfs(int64_t n, const uint8_t* A, const int64_t* rows, int64_t nrows, uint8_t* R,
           int64_t* hist) {
  if (n < 0) return 3;
  csr g, gt;
  if (build_csr(n, A, 0, &g)) return 2;
  if (build_csr(n, A, 1, &gt)) { free_csr(&g); return 2; }
  int64_t ns = rows ? nrows : n;
  if (hist) memset(hist, 0, (size_t)(n + 2) * sizeof(int64_t));
  int fail = 0;
#pragma omp parallel
  {
    int64_t* dist = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t* queue = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    int64_t* h = (int64_t*)calloc((size_t)(n + 2), sizeof(int64_t));
    if (!dist || !queue || !h) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 8)
      for (int64_t si = 0; si < ns; ++si) {
        int64_t s = rows ? rows[si] : si;
        for (int64_t i = 0; i < n; ++i) dist[i] = -1;
        int64_t head = 0, tail = 0;
        dist[s] = 0;
        queue[tail++] = (int32_t)s;
        while (head < tail) {
          int32_t u = queue[head++];
          for (int64_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
            int32_t v = g.idx[e];
            if (dist[v] < 0) { dist[v] = dist[u] + 1; queue[tail++] = v; }
          }
        }
        /* shortest cycle through s: one edge from a reachable predecessor */
        int64_t self = -1;
        for (int64_t e = gt.ptr[s]; e < gt.ptr[s + 1]; ++e) {
          int32_t p = gt.idx[e];
          if (dist[p] >= 0 && (self < 0 || dist[p] + 1 < self)) self = dist[p] + 1;
        }
        uint8_t* rrow = R ? R + si * n : NULL;
        for (int64_t t = 0; t < n; ++t) {
          int64_t d = (t == s) ? self : dist[t];
          if (rrow) rrow[t] = (uint8_t)(d >= 1);
          if (d >= 1) h[d]++;
        }
      }
      if (hist) {
#pragma omp critical
        for (int64_t i = 0; i < n + 2; ++i) hist[i] += h[i];
      }
    }
    free(dist); free(queue); free(h);
  }
  free_csr(&g); free_csr(&gt);
  return fail ? 2 : 0;
}

/*
 * Same generation, semi-naive.  Round 1 derives r2 from diag: S_1 = Delta_1 = I
 * over all n constants.  Round k+1 applies the recursive rule to the facts
 * new in round k:
 *   Delta_{k+1} = { (x, w) : P(x, y), Delta_k(y, z), P(w, z) } \ S_k.
 * Computed as Y = Delta_k P^T  (Y(y) = OR_{z in Delta_k(y)} col_z(P)),
 * then Z(x) = OR_{y in succ_P(x)} Y(y), then Delta_{k+1} = Z \ S_k.
 */
int or_sg_seminaive(int64_t n, const uint8_t* P, uint8_t* S, int64_t* ones, int64_t maxsteps,
                    int64_t* iters) {
  if (n < 0 || maxsteps < 0) return 3;
  int64_t w = nwords(n);
  csr g;
  if (build_csr(n, P, 0, &g)) return 2;
  /* PT(z) = { w : P(w, z) } as a bitset row */
  word* PT = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  word* T = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  word* D = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  word* Y = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  word* Dn = (word*)calloc((size_t)(n * w + 1), sizeof(word));
  if (!PT || !T || !D || !Y || !Dn) {
    free(PT); free(T); free(D); free(Y); free(Dn); free_csr(&g);
    return 2;
  }
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = 0; b < n; ++b)
      if (P[a * n + b]) set_bit(PT + b * w, a);
  int rc = 0;
  int64_t k = 0;
  if (ones) ones[0] = 0;
  if (maxsteps > 0 && n > 0) {
    for (int64_t i = 0; i < n; ++i) { set_bit(T + i * w, i); set_bit(D + i * w, i); }
    k = 1;
    if (ones) ones[1] = n;
    for (;;) {
      if (k == maxsteps) { rc = 1; break; }
#pragma omp parallel for schedule(dynamic, 16)
      for (int64_t y = 0; y < n; ++y) {
        word* yr = Y + y * w;
        memset(yr, 0, (size_t)w * sizeof(word));
        const word* dr = D + y * w;
        for (int64_t z = 0; z < n; ++z)
          if (get_bit(dr, z)) {
            const word* pz = PT + z * w;
            for (int64_t q = 0; q < w; ++q) yr[q] |= pz[q];
          }
      }
      int64_t delta = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : delta)
      for (int64_t x = 0; x < n; ++x) {
        word* dst = Dn + x * w;
        memset(dst, 0, (size_t)w * sizeof(word));
        for (int64_t e = g.ptr[x]; e < g.ptr[x + 1]; ++e) {
          const word* src = Y + (int64_t)g.idx[e] * w;
          for (int64_t q = 0; q < w; ++q) dst[q] |= src[q];
        }
        word* t = T + x * w;
        for (int64_t q = 0; q < w; ++q) { dst[q] &= ~t[q]; t[q] |= dst[q]; }
        delta += popcount_row(dst, w);
      }
      word* tmp = D; D = Dn; Dn = tmp;
      ++k;
      if (ones) ones[k] = ones[k - 1] + delta;
      if (delta == 0) break;
    }
  } else if (n == 0 && maxsteps > 0) {
    k = 1;
    if (ones) ones[1] = 0;
  }
  if (iters) *iters = k;
  if (S) bits_to_dense(n, T, S);
  free(PT); free(T); free(D); free(Y); free(Dn); free_csr(&g);
  return rc;
}
