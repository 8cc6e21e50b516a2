// eps_solve.hip -- the epsilon form of Sec. 4 (Proposition 1, Theorem 1):
// X = (I - eps A)^-1 eps A in fp64, then R = [X > 0].
//
// Method: block Gauss-Jordan elimination without pivoting on the augmented
// matrix W = [ I - eps A | eps A ]  (Np x 2Np, row-major), in pivot panels
// p of 512 rows and columns (T = the columns right of the panel):
//   D^-1 = W[p, p]^-1             (the same elimination at block size 128 on
//                                  [W[p, p] | I]; 128 x 128 blocks inverted
//                                  by Gauss-Jordan in one workgroup)
//   Y = D^-1 W[p, T];  W[q, T] -= W[q, p] Y for every row q outside p;
//   W[p, T] = Y                    (fp64 MFMA products)
// Columns left of T are never touched again (they would hold the identity
// and zeros), so after the last panel the right half of W is X.  About
// 3 Np^3 flops, almost all in one full-height product per panel.
//
// Why no pivoting: M = I - eps A has unit diagonal and off-diagonal entries
// <= 0 with eps * (row sum of A) < 1 (Lemma 1's eps bound), so M is a
// strictly diagonally dominant M-matrix; its Schur complements stay
// M-matrices, their inverses are entrywise >= 0, and every update above adds
// terms of one sign to the off-diagonal and right-hand-side entries (rows
// above the diagonal block hold entries <= 0 in the columns being
// eliminated, just like the rows below).  Exact
// zeros therefore stay exactly zero and positive entries never cancel:
// thresholding at > 0 is exact except where a true value underflows fp64
// (it is at least eps^L for a shortest path of length L, by the footnote to
// Lemma 2).  Denormals are kept.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "eps_solve.h"

namespace dl {

constexpr int NB = 128;  // block size of the elimination

// ----------------------------------------------------------------- fp64 MFMA GEMM
// D = A * B (cmode 0), D = C - A * B (cmode 1) or D = C + A * B (cmode 2);
// A: M x K, B: K x N, C/D: M x N, row-major.  128 x 128 output tiles, 4 waves
// of 64 x 64 (v_mfma_f64_16x16x4f64), K slices of 16 fetched straight into a
// 4-slot LDS ring (global_load_lds, three slices in flight).  With cmode 1
// or 2 the accumulators start from C (negated for cmode 1, and the result
// negated back on the way out: both exact), so C is read once at the start of
// the tile and D written once at the end.  Row tiles at or after
// skip_tile are shifted down by skip_count, which leaves out the row tiles
// skip_tile .. skip_tile + skip_count - 1 (the pivot rows of an elimination
// step; skip_tile -1 = none).  D may alias C
// (every element is read and written by the same lane); D may also alias B
// when M = K = 128 and cmode = 0 (each workgroup reads its whole B column panel
// before writing it).  A must not overlap D.
struct GemmArgs {
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  const double* C; int64_t ldc;
  double* D; int64_t ldd;
  int M, N, K;      // M counts the rows computed (without the skipped tiles)
  int cmode;
  int skip_tile;
  int skip_count = 1;
};

// Output coordinate of accumulator element `item` of lane `lane` for
// v_mfma_f64_16x16x4f64 (gfx950), as measured on the device.
__device__ inline void f64_acc_coord(int lane, int item, int& r, int& c) {
  r = (lane >> 4) + 4 * item;
  c = lane & 15;
}

// LDS of one slice: the A slice (128 rows x 16 doubles, 128-byte rows; the
// 16-byte chunk c of row r at position c ^ ((r >> 1) & 7)) then the B slice
// (16 k-rows x 128 doubles, 1 KB rows; chunk c of k-row k at c ^ 8 (k & 1)).
// Either way the 32 lanes that one ds_read_b64 pass serves (two k values x
// 16 rows or columns) hit 64 distinct banks.
constexpr int kDgemmStages = 4;
constexpr int kDgemmSliceBytes = 2 * 128 * 16 * 8;
constexpr unsigned kDgemmLds = kDgemmStages * kDgemmSliceBytes;  // 128 KB: one update workgroup per CU

// s_waitcnt with vmcnt = N and no wait on the other counters
template <int N>
__device__ inline void dgemm_wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

__global__ void __launch_bounds__(256) k_dgemm(GemmArgs g) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int tiles_m = g.M / 128;
  // column-major walk over tiles keeps one B column panel hot across rows
  int tm = blockIdx.x % tiles_m;
  const int tn = blockIdx.x / tiles_m;
  if (g.skip_tile >= 0 && tm >= g.skip_tile) tm += g.skip_count;
  const int m0 = tm * 128, n0 = tn * 128;

  // Each wave issues 8 of a slice's 32 one-KB direct-to-LDS instructions:
  // A instruction a = wave + 4 jj covers rows 8a .. 8a + 7 (lane l: row
  // 8a + l / 8, LDS chunk l % 8), B instruction b = wave + 4 jj is k-row b
  // (lane l: LDS chunk l).
  const double* asrc[4];
  const double* bsrc[4];
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int a = wave + 4 * jj;
    const int row = 8 * a + (lane >> 3);
    asrc[jj] = g.A + (int64_t)(m0 + row) * g.lda + 2 * ((lane & 7) ^ ((row >> 1) & 7));
    bsrc[jj] = g.B + (int64_t)a * g.ldb + n0 + 2 * (lane ^ (8 * (a & 1)));
  }
  auto issue = [&](int kt) {
    uint8_t* stage = lds + (kt % kDgemmStages) * kDgemmSliceBytes;
    const int k0 = kt * 16;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(asrc[jj] + k0),
                                       (__attribute__((address_space(3))) void*)(stage + (wave + 4 * jj) * 1024),
                                       16, 0, 0);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(bsrc[jj] + (int64_t)k0 * g.ldb),
                                       (__attribute__((address_space(3))) void*)(stage + 16384 + (wave + 4 * jj) * 1024),
                                       16, 0, 0);
  };

  // fragment reads: lane (g4, r16) = (lane / 16, lane % 16) supplies
  // A[row r16][k g4] and B[k g4][column r16] of each 16 x 16 x 4 product
  const int g4 = lane >> 4, r16 = lane & 15;
  auto frags = [&](const uint8_t* st, int kk, double* af, double* bf) {
    const int k = kk + g4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 64 + i * 16 + r16;
      af[i] = *(const double*)(st + r * 128 + (((k >> 1) ^ ((r >> 1) & 7)) << 4) + ((k & 1) << 3));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = wn * 64 + j * 16 + r16;
      bf[j] = *(const double*)(st + 16384 + k * 1024 + (((n >> 1) ^ (8 * (k & 1))) << 4) + ((n & 1) << 3));
    }
  };

  const int nk = g.K / 16;
#pragma unroll
  for (int s0 = 0; s0 < kDgemmStages - 1; ++s0)
    if (s0 < nk) issue(s0);

  // the accumulators from C while the first slices are in flight
  v4d acc[4][4];
  const double csgn = g.cmode == 1 ? -1.0 : 1.0;
  if (g.cmode) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int r, c;
          f64_acc_coord(lane, v, r, c);
          acc[i][j][v] = csgn * g.C[(int64_t)(m0 + wm * 64 + i * 16 + r) * g.ldc + n0 + wn * 64 + j * 16 + c];
        }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  }

  for (int kt = 0; kt < nk; ++kt) {
    // slice kt has landed once at most the later slices' instructions
    // (8 per slice) are outstanding; the barrier extends that to every wave
    // and retires every read of slot (kt - 1) % 4, refilled below
    const int later = (kt + 2 < nk ? kt + 2 : nk - 1) - kt;
    if (later >= 2) dgemm_wait_vmcnt<16>();
    else if (later == 1) dgemm_wait_vmcnt<8>();
    else dgemm_wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (kt + kDgemmStages - 1 < nk) issue(kt + kDgemmStages - 1);
    const uint8_t* st = lds + (kt % kDgemmStages) * kDgemmSliceBytes;
    double af[2][4], bf[2][4];
    frags(st, 0, af[0], bf[0]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < 3) frags(st, 4 * (q + 1), af[(q + 1) & 1], bf[(q + 1) & 1]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[q & 1][i], bf[q & 1][j], acc[i][j], 0, 0, 0);
    }
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r, c;
        f64_acc_coord(lane, v, r, c);
        const int64_t row = m0 + wm * 64 + i * 16 + r, col = n0 + wn * 64 + j * 16 + c;
        g.D[row * g.ldd + col] = csgn * acc[i][j][v];
      }
}

static hipError_t dgemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.M % 128 || g.N % 128 || g.K % 16) return hipErrorInvalidValue;
  const int grid = (g.M / 128) * (g.N / 128);
  hipLaunchKernelGGL(k_dgemm, dim3(grid), dim3(256), kDgemmLds, s, g);
  return hipGetLastError();
}

// ----------------------------------------------------------------- diagonal block inverse
// In-place Gauss-Jordan inversion of the NB x NB block at W (ld), written to
// Dinv (ld NB), with pivot blocks of PB rows and columns S = p .. p + PB - 1
// (NB / PB steps of one barrier each).  1024 threads; thread t owns row t / 8
// and the 16 contiguous columns 16 (t % 8) + m.  A step broadcasts the rows
// and columns of S through LDS (double buffered); every thread inverts the
// PB x PB pivot block P = a[S][S] itself (Gauss-Jordan in registers) and
// updates its 16 entries:
//   rows of S:   a[S][j] = P^-1 a[S][j]  (j not in S),   a[S][S] = P^-1
//   other rows:  f = a[i][S] P^-1;  a[i][j] -= f a[S][j]  (j not in S),
//                a[i][S] = -f
// which is PB single-pivot steps done at once.  Signs: the block is a
// strictly diagonally dominant M-matrix, so P^-1 >= 0 entrywise and, as for
// single pivots, every update adds terms of one sign to each off-diagonal
// entry (columns already pivoted hold entries >= 0, the others <= 0), so
// zeros stay exact and nothing cancels.  The kernel runs beside the
// trailing update (another stream): PB = 2 keeps it within the registers
// that one resident update workgroup leaves free on a compute unit.
constexpr int PB = 2;
__global__ void __launch_bounds__(1024) k_block_inverse(const double* W, int64_t ld, double* Dinv) {
  // the next panel's inverse shares its compute unit with a trailing-update
  // workgroup and is the longer chain in the late panels: its waves issue
  // first (0.2-0.3 ms per N = 8192 solve)
  __builtin_amdgcn_s_setprio(3);
  __shared__ __attribute__((aligned(16))) double rowbuf[2][PB][NB];
  __shared__ double colbuf[2][PB][NB];
  const int t = threadIdx.x;
  const int i = t >> 3, j0 = (t & 7) * 16;
  double a[16];
#pragma unroll
  for (int m = 0; m < 16; m += 2) {
    const double2 v = *(const double2*)(W + (int64_t)i * ld + j0 + m);
    a[m] = v.x;
    a[m + 1] = v.y;
  }
  for (int p = 0; p < NB; p += PB) {
    const int b = (p / PB) & 1;
    const bool owns_cols = (p >> 4) == (t & 7);  // columns p .. p + PB - 1 are among this thread's 16
    const int pc = p & 15;                       // their position in a[]
    const int r_in = i - p;                      // row of S held by this thread, if 0 <= r_in < PB
    const bool in_s = r_in >= 0 && r_in < PB;
    if (in_s) {
#pragma unroll
      for (int m = 0; m < 16; m += 2) *(double2*)&rowbuf[b][r_in][j0 + m] = make_double2(a[m], a[m + 1]);
    }
    if (owns_cols) {
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        double v = a[0];
#pragma unroll
        for (int m = 1; m < 16; ++m) v = (m == pc + k) ? a[m] : v;
        colbuf[b][k][i] = v;
      }
    }
    __syncthreads();
    // P^-1 by Gauss-Jordan without pivoting (every thread, same result)
    double q[PB][PB];
#pragma unroll
    for (int r = 0; r < PB; ++r)
#pragma unroll
      for (int c = 0; c < PB; ++c) q[r][c] = rowbuf[b][r][p + c];
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      const double inv = 1.0 / q[k][k];
#pragma unroll
      for (int r = 0; r < PB; ++r) {
        if (r == k) continue;
        const double f = q[r][k] * inv;
#pragma unroll
        for (int c = 0; c < PB; ++c)
          if (c != k) q[r][c] = __builtin_fma(-f, q[k][c], q[r][c]);
        q[r][k] = -f;
      }
#pragma unroll
      for (int c = 0; c < PB; ++c) q[k][c] = (c == k) ? inv : q[k][c] * inv;
    }
    // the multipliers of this thread's row: f = a[i][S] P^-1 (other rows),
    // or row r_in of P^-1 (rows of S)
    double f[PB];
    if (!in_s) {
#pragma unroll
      for (int c = 0; c < PB; ++c) f[c] = 0.0;
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        const double ck = colbuf[b][k][i];
#pragma unroll
        for (int c = 0; c < PB; ++c) f[c] = __builtin_fma(ck, q[k][c], f[c]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        f[c] = q[0][c];
#pragma unroll
        for (int r = 1; r < PB; ++r) f[c] = (r == r_in) ? q[r][c] : f[c];
      }
    }
    // other rows: a -= f a[S][.];  rows of S: a = f a[S][.] (sign and start differ)
    const double sg = in_s ? 1.0 : -1.0;
#pragma unroll
    for (int m = 0; m < 16; m += 2) {
      double2 acc = in_s ? make_double2(0.0, 0.0) : make_double2(a[m], a[m + 1]);
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        const double2 r = *(const double2*)&rowbuf[b][c][j0 + m];
        acc.x = __builtin_fma(sg * f[c], r.x, acc.x);
        acc.y = __builtin_fma(sg * f[c], r.y, acc.y);
      }
      a[m] = acc.x;
      a[m + 1] = acc.y;
    }
    if (owns_cols) {  // the columns of S: -f (other rows) or P^-1 (rows of S)
#pragma unroll
      for (int m = 0; m < 16; ++m)
#pragma unroll
        for (int c = 0; c < PB; ++c)
          if (m == pc + c) a[m] = sg * f[c];
    }
  }
#pragma unroll
  for (int m = 0; m < 16; m += 2) *(double2*)&Dinv[i * NB + j0 + m] = make_double2(a[m], a[m + 1]);
}

// ----------------------------------------------------------------- setup / copy / emit
// W[i][j] = [i == j] - eps b_ij  and  W[i][Np + j] = eps c_ij, padded rows and
// columns carry the identity and zeros.
__global__ void __launch_bounds__(256) k_eps_init(const uint8_t* B, int64_t ldb, const uint8_t* C, int64_t ldc,
                                                  int n, int Np, double eps, double* W) {
  const int i = blockIdx.y;
  const int64_t ld = 2 * (int64_t)Np;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < Np; j += gridDim.x * 256) {
    const bool in = i < n && j < n;
    const double b = (in && B[(int64_t)i * ldb + j] != 0) ? 1.0 : 0.0;
    const double c = (in && C[(int64_t)i * ldc + j] != 0) ? 1.0 : 0.0;
    W[i * ld + j] = (i == j ? 1.0 : 0.0) - eps * b;
    W[i * ld + Np + j] = eps * c;
  }
}

// R = [X > 0] (and X itself when asked for), plus the smallest positive
// entry of X: its bits go into *minpos by an unsigned atomic minimum (positive
// doubles order like their bit patterns), one per workgroup.  A fixed grid
// walks the rows, so the atomics stay few.
constexpr int kEmitBlocks = 1024;
__global__ void __launch_bounds__(256)
k_eps_emit(const double* W, int Np, int n, uint8_t* R, int64_t ldr, double* X, int64_t ldx,
           unsigned long long* minpos) {
  __shared__ unsigned long long red[4];
  const int64_t ld = 2 * (int64_t)Np;
  unsigned long long m = ~0ull;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    for (int j = threadIdx.x; j < n; j += 256) {
      const double x = W[i * ld + Np + j];
      R[(int64_t)i * ldr + j] = x > 0.0 ? 1 : 0;
      if (X) X[(int64_t)i * ldx + j] = x;
      if (x > 0.0) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(x);
        m = b < m ? b : m;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long v = __shfl_xor(m, o);
    m = v < m ? v : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) m = red[w] < m ? red[w] : m;
    if (m != ~0ull) atomicMin(minpos, m);
  }
}

__global__ void k_set_word(unsigned long long* p, unsigned long long v) { *p = v; }

// ----------------------------------------------------------------- driver
hipError_t eps_kernels_init() {
  return hipFuncSetAttribute((const void*)k_dgemm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDgemmLds);
}

int64_t eps_padded_size(int64_t n) { return n <= 0 ? 0 : ((n + NB - 1) / NB) * NB; }

void eps_free(EpsWorkspace* ws) {
  if (ws->buf) (void)hipFree(ws->buf);
  ws->buf = nullptr;
  ws->size = 0;
}

void eps_release(EpsWorkspace* ws) {
  eps_free(ws);
  for (auto& e : ws->ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (ws->side) (void)hipStreamDestroy(ws->side);
  if (ws->work) (void)hipStreamDestroy(ws->work);
  ws->side = ws->work = nullptr;
}

static hipError_t ensure(EpsWorkspace* ws, size_t budget_left, size_t need, const char* what, std::string* err) {
  if (need <= ws->size) return hipSuccess;
  if (budget_left && need > budget_left) {
    *err = std::string(what) + " workspace of " + std::to_string(need) + " bytes exceeds the budget";
    return hipErrorOutOfMemory;
  }
  eps_free(ws);
  hipError_t e = hipMalloc(&ws->buf, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ws->buf = nullptr;
    *err = "hipMalloc of " + std::to_string(need) + " bytes for the " + what + " failed";
    return hipErrorOutOfMemory;
  }
  ws->size = need;
  return hipSuccess;
}

#define EPS_CK(x, what)            \
  do {                             \
    hipError_t e_ = (x);           \
    if (e_ != hipSuccess) {        \
      *err = what;                 \
      return e_;                   \
    }                              \
  } while (0)

// Gauss-Jordan elimination, block size NB, of the Ns x Ns system in the left
// part of V (row stride ldv, Ns + right-hand-side columns); afterwards the
// columns Ns .. ldv of V hold the solution.  Used on the P x 2P panel
// systems [D | I] below, whose right half becomes D^-1.  Dinv: NB x NB.
static hipError_t gj_blocks(double* V, int64_t Ns, int64_t ldv, double* Dinv, hipStream_t s, std::string* err) {
  const int nblk = (int)(Ns / NB);
  for (int k = 0; k < nblk; ++k) {
    const int64_t K0 = (int64_t)k * NB;
    const int cols = (int)(ldv - K0 - NB);
    hipLaunchKernelGGL(k_block_inverse, dim3(1), dim3(1024), 0, s, (const double*)(V + K0 * ldv + K0), ldv, Dinv);
    EPS_CK(hipGetLastError(), "block inverse");
    GemmArgs rp{Dinv, NB, V + K0 * ldv + K0 + NB, ldv, nullptr, 0, V + K0 * ldv + K0 + NB, ldv, NB, cols, NB, 0, -1};
    EPS_CK(dgemm(rp, s), "row panel product");
    if (nblk > 1) {
      GemmArgs up{V + K0, ldv, V + K0 * ldv + K0 + NB, ldv, V + K0 + NB, ldv, V + K0 + NB, ldv,
                  (int)(Ns - NB), cols, NB, 1, k};
      EPS_CK(dgemm(up, s), "elimination update");
    }
  }
  return hipSuccess;
}

// V = [ W[r0 : r0 + P, r0 : r0 + P] | I_P ]  (P x 2P)
__global__ void __launch_bounds__(256)
k_panel_copy(const double* W, int64_t ldw, int64_t r0, int P, double* V) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < 2 * P; j += gridDim.x * 256)
    V[(int64_t)i * 2 * P + j] = j < P ? W[(r0 + i) * ldw + r0 + j] : (j - P == i ? 1.0 : 0.0);
}

// W[r0 + i, c0 + j] = Y[i, j] for i < P, j < n (Y row stride ldy)
__global__ void __launch_bounds__(256)
k_rows_store(const double* Y, int64_t ldy, int P, int64_t n, double* W, int64_t ldw, int64_t r0, int64_t c0) {
  const int i = blockIdx.y;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    W[(r0 + i) * ldw + c0 + j] = Y[i * ldy + j];
}

// Block Gauss-Jordan elimination of the Ns x Ns system held in the left part
// of W (Ns rows, row stride ldw >= Ns + right-hand-side columns); afterwards
// columns Ns .. ldw of W hold the solution.  Ns is a multiple of NB.
// Pivot panels of P = kPanel rows and columns: with D = W[p, p] and T the
// columns right of the panel,
//   Y = D^-1 W[p, T];   W[q, T] -= W[q, p] Y for every row q outside p;
//   W[p, T] = Y,
// so the trailing matrix is read and written once per panel with K = P in
// the update product (fp64 MFMA; the update is bound by that traffic at
// small K).  D^-1 comes from gj_blocks on [D | I].  Look-ahead: the update
// of the next panel's columns runs first; the next D is then final and is
// inverted on the side stream while the rest of the update runs.
constexpr int kPanel = 4 * NB;

// The elimination's two streams (default priority): the work stream takes
// the updates, the side stream the look-ahead panel inverse.
static hipError_t ensure_streams(EpsWorkspace* ws, std::string* err) {
  if (ws->side) return hipSuccess;
  EPS_CK(hipStreamCreateWithFlags(&ws->side, hipStreamNonBlocking), "side stream");
  EPS_CK(hipStreamCreateWithFlags(&ws->work, hipStreamNonBlocking), "work stream");
  for (auto& e : ws->ev) EPS_CK(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  return hipSuccess;
}

static hipError_t gj_eliminate(EpsWorkspace* ws, double* W, int64_t Ns, int64_t ldw, double* scratch, hipStream_t s,
                               bool timing, std::vector<std::pair<hipEvent_t, hipEvent_t>>* evs, std::string* err) {
  // the caller's stream s hands over to the work stream and takes it back
  EPS_CK(ensure_streams(ws, err), *err);
  EPS_CK(hipEventRecord(ws->ev[2], s), "event");
  EPS_CK(hipStreamWaitEvent(ws->work, ws->ev[2], 0), "wait");
  const hipStream_t caller = s;
  s = ws->work;
  auto timed = [&](const GemmArgs& g) -> hipError_t {
    hipEvent_t ea = nullptr, eb = nullptr;
    if (timing && hipEventCreate(&ea) == hipSuccess && hipEventCreate(&eb) == hipSuccess) (void)hipEventRecord(ea, s);
    hipError_t e = dgemm(g, s);
    if (ea && eb) {
      (void)hipEventRecord(eb, s);
      evs->push_back({ea, eb});
    }
    return e;
  };
  // scratch: V[2] (kPanel x 2 kPanel each), Dinv (NB x NB), Y (kPanel x ldw)
  double* V[2] = {scratch, scratch + (size_t)2 * kPanel * kPanel};
  double* Dinv = V[1] + (size_t)2 * kPanel * kPanel;
  double* Y = Dinv + (size_t)NB * NB;
  auto invert = [&](int64_t r0, int P, double* v, hipStream_t st) -> hipError_t {
    hipLaunchKernelGGL(k_panel_copy, dim3((unsigned)((2 * P + 255) / 256), (unsigned)P), dim3(256), 0, st,
                       (const double*)W, ldw, r0, P, v);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return gj_blocks(v, P, 2 * P, Dinv, st, err);  // panel inversions never overlap
  };
  int P = (int)std::min<int64_t>(kPanel, Ns);
  EPS_CK(invert(0, P, V[0], s), "panel inverse");
  int t = 0;
  for (int64_t K0 = 0; K0 < Ns; K0 += P, ++t) {
    P = (int)std::min<int64_t>(kPanel, Ns - K0);
    const double* Dp = V[t & 1] + P;  // D^-1, row stride 2P
    const int64_t T0 = K0 + P;
    const int nT = (int)(ldw - T0);
    // Y = D^-1 W[p, T]
    GemmArgs gy{Dp, 2 * P, W + K0 * ldw + T0, ldw, nullptr, 0, Y, ldw, P, nT, P, 0, -1};
    EPS_CK(dgemm(gy, s), "panel row product");
    const bool ahead = T0 < Ns;
    const int Pn = ahead ? (int)std::min<int64_t>(kPanel, Ns - T0) : 0;
    const int first = ahead ? Pn : nT;
    if (Ns > P) {
      GemmArgs ua{W + K0, ldw, Y, ldw, W + T0, ldw, W + T0, ldw, (int)(Ns - P), first, P, 1, (int)(K0 / 128)};
      ua.skip_count = P / 128;
      EPS_CK(timed(ua), "elimination update");
    }
    if (ahead) {
      EPS_CK(hipEventRecord(ws->ev[0], s), "event");
      EPS_CK(hipStreamWaitEvent(ws->side, ws->ev[0], 0), "wait");
      EPS_CK(invert(T0, Pn, V[(t + 1) & 1], ws->side), "panel inverse");
      EPS_CK(hipEventRecord(ws->ev[1], ws->side), "event");
      if (nT > Pn) {
        GemmArgs ub{W + K0, ldw, Y + Pn, ldw, W + T0 + Pn, ldw, W + T0 + Pn, ldw, (int)(Ns - P), nT - Pn, P, 1,
                    (int)(K0 / 128)};
        ub.skip_count = P / 128;
        EPS_CK(timed(ub), "elimination update");
      }
    }
    // the pivot rows take Y
    hipLaunchKernelGGL(k_rows_store, dim3((unsigned)((nT + 255) / 256), (unsigned)P), dim3(256), 0, s,
                       (const double*)Y, ldw, P, (int64_t)nT, W, ldw, K0, T0);
    EPS_CK(hipGetLastError(), "pivot rows");
    if (ahead) EPS_CK(hipStreamWaitEvent(s, ws->ev[1], 0), "wait");
  }
  EPS_CK(hipEventRecord(ws->ev[3], s), "event");
  EPS_CK(hipStreamWaitEvent(caller, ws->ev[3], 0), "wait");
  return hipSuccess;
}

// Scratch doubles gj_eliminate needs beyond W.
static size_t gj_scratch_doubles(int64_t ldw) {
  return (size_t)4 * kPanel * kPanel + (size_t)NB * NB + (size_t)kPanel * ldw;
}

hipError_t eps_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* B, int64_t ldb,
                     const uint8_t* C, int64_t ldc, double eps, uint8_t* R, int64_t ldr, double* X_out,
                     int64_t ldx, hipStream_t s, bool timing, double* trailing_ms, int64_t* trailing_launches,
                     double* min_positive, std::string* err) {
  *trailing_ms = 0.0;
  *trailing_launches = 0;
  const int64_t Np = eps_padded_size(n);
  const int64_t ldw = 2 * Np;
  const size_t wbytes = (size_t)Np * ldw * sizeof(double);
  const size_t dbytes = gj_scratch_doubles(ldw) * sizeof(double);
  EPS_CK(ensure(ws, budget_left, wbytes + dbytes + 256, "epsilon-solve", err), *err);
  double* W = (double*)ws->buf;
  double* Dinv = W + (size_t)Np * ldw;
  unsigned long long* minpos = (unsigned long long*)((char*)ws->buf + wbytes + dbytes);
  hipLaunchKernelGGL(k_set_word, dim3(1), dim3(1), 0, s, minpos, ~0ull);
  EPS_CK(hipGetLastError(), "epsilon init");

  hipLaunchKernelGGL(k_eps_init, dim3((unsigned)((Np + 255) / 256), (unsigned)Np), dim3(256), 0, s, B, ldb, C, ldc,
                     (int)n, (int)Np, eps, W);
  EPS_CK(hipGetLastError(), "epsilon init");
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
  hipError_t e = gj_eliminate(ws, W, Np, ldw, Dinv, s, timing, &evs, err);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_eps_emit, dim3((unsigned)std::min<int64_t>(n, kEmitBlocks)), dim3(256), 0, s, W, (int)Np,
                       (int)n, R, ldr, X_out, ldx, minpos);
    e = hipGetLastError();
    if (e != hipSuccess) *err = "threshold";
  }
  unsigned long long mp = ~0ull;
  if (e == hipSuccess) {
    e = hipMemcpyAsync(&mp, minpos, sizeof mp, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) *err = "smallest positive entry read-back";
  }
  if (e == hipSuccess) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) *err = "epsilon solve sync";
  }
  if (min_positive) {
    double v = INFINITY;
    if (mp != ~0ull) memcpy(&v, &mp, sizeof v);
    *min_positive = v;
  }
  for (auto& p : evs) {
    float t = 0.f;
    if (e == hipSuccess && hipEventElapsedTime(&t, p.first, p.second) == hipSuccess) {
      *trailing_ms += t;
      *trailing_launches += 1;
    }
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  return e;
}

// ----------------------------------------------------------------- stacked tail-recursive system
// W = [ I - E BB | E AA ] for the heads h = 0 .. M-1 of one layer (Ns = M Np
// rows, ldw = Ns + Np): block (h, j) of BB is the int8 0/1 matrix B[h][j]
// (null = zero), block h of AA is A[h], E = diag(eps_h) row-block-wise.
__global__ void __launch_bounds__(256) k_stack_init(StackDesc d, int64_t Ns, int64_t ldw, double* W) {
  const int64_t i = blockIdx.y;
  const int h = (int)(i / d.Np), ii = (int)(i % d.Np);
  const double eps = d.eps[h];
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < ldw; j += (int64_t)gridDim.x * 256) {
    double v;
    if (j < Ns) {
      const int jb = (int)(j / d.Np), jj = (int)(j % d.Np);
      const int8_t* b = d.B[h][jb];
      const double bij = (b && b[(int64_t)ii * d.Np + jj] != 0) ? 1.0 : 0.0;
      v = (i == j ? 1.0 : 0.0) - eps * bij;
    } else {
      const int8_t* a = d.A[h];
      const int jj = (int)(j - Ns);
      v = (a && a[(int64_t)ii * d.Np + jj] != 0) ? eps : 0.0;
    }
    W[i * ldw + j] = v;
  }
}

// R[h] = [X_h > 0] as int8 0/1 (Np x Np), counting the ones of each head.
__global__ void __launch_bounds__(256) k_stack_emit(StackDesc d, int64_t Ns, int64_t ldw, const double* W) {
  const int64_t i = blockIdx.y;
  const int h = (int)(i / d.Np), ii = (int)(i % d.Np);
  int c = 0;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < d.Np; j += gridDim.x * 256) {
    const int8_t v = W[i * ldw + Ns + j] > 0.0 ? 1 : 0;
    d.R[h][(int64_t)ii * (d.ldr ? d.ldr : d.Np) + j] = v;
    c += v;
  }
  if (!d.cnt) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = red[0] + red[1] + red[2] + red[3];
    if (t) atomicAdd(d.cnt + h, (unsigned long long)t);
  }
}

hipError_t stacked_solve(EpsWorkspace* ws, size_t budget_left, const StackDesc& d, hipStream_t s, std::string* err) {
  if (d.M < 1 || d.M > kMaxStack || d.Np % NB) {
    *err = "bad stacked system";
    return hipErrorInvalidValue;
  }
  const int64_t Ns = (int64_t)d.M * d.Np;
  const int64_t ldw = Ns + d.Np;
  const size_t wbytes = (size_t)Ns * ldw * sizeof(double);
  const size_t dbytes = gj_scratch_doubles(ldw) * sizeof(double);
  EPS_CK(ensure(ws, budget_left, wbytes + dbytes, "stacked linear solve", err), *err);
  double* W = (double*)ws->buf;
  double* Dinv = W + (size_t)Ns * ldw;
  hipLaunchKernelGGL(k_stack_init, dim3((unsigned)((ldw + 255) / 256), (unsigned)Ns), dim3(256), 0, s, d, Ns, ldw, W);
  EPS_CK(hipGetLastError(), "stacked init");
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
  EPS_CK(gj_eliminate(ws, W, Ns, ldw, Dinv, s, false, &evs, err), *err);
  hipLaunchKernelGGL(k_stack_emit, dim3((unsigned)((d.Np + 255) / 256), (unsigned)Ns), dim3(256), 0, s, d, Ns, ldw,
                     (const double*)W);
  EPS_CK(hipGetLastError(), "stacked threshold");
  return hipSuccess;
}

// ----------------------------------------------------------------- two-sided (Stein) equations
// X = Q + B X C with B, C, Q >= 0 and a convergent series, solved by Smith's
// doubling in fp64:
//   X_0 = Q,  B_0 = B,  C_0 = C,
//   X_{j+1} = X_j + B_j X_j C_j,  B_{j+1} = B_j B_j,  C_{j+1} = C_j C_j,
// so X_j = sum_{m < 2^j} B^m Q C^m.  Every term is >= 0, so the zero pattern
// of X_j is exact: it is the 2^j-th iterate of the Boolean series
// Y' = [Q + B Y C] from Y = 0.  When a doubling leaves the number of positive
// entries unchanged, that series has repeated (it is monotone), so the
// pattern is the least model.  When the real solution is wanted as well,
// doublings go on until one also leaves every fp64 value unchanged (the
// increments shrink doubly exponentially, so the truncated series is then
// within rounding of the limit).  A Schur-based Sylvester solver would
// cancel terms and lose the exact zero pattern.  For the same-generation
// form C = B^T, which is kept as the transpose of B instead of a product.
__global__ void __launch_bounds__(256)
k_f64_from_bytes(const uint8_t* src, int64_t ld, int n, int Np, double scale, int identity, double* dst) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < Np; j += gridDim.x * 256) {
    double v = 0.0;
    if (i < n && j < n) v = identity ? (i == j ? scale : 0.0) : (src[(int64_t)i * ld + j] != 0 ? scale : 0.0);
    dst[(int64_t)i * Np + j] = v;
  }
}

__global__ void __launch_bounds__(256) k_transpose_f64(const double* src, double* dst, int Np) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
#pragma unroll
  for (int r = ty; r < 32; r += 8) tile[r][tx] = src[(int64_t)(by + r) * Np + bx + tx];
  __syncthreads();
#pragma unroll
  for (int r = ty; r < 32; r += 8) dst[(int64_t)(bx + r) * Np + by + tx] = tile[tx][r];
}

// Block sums of per-thread counts into out[0..K): one atomic per workgroup and counter.
template <int K>
__device__ inline void block_count(int (&c)[K], unsigned long long* out) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c[k] += __shfl_xor(c[k], off, 64);
  __shared__ int red[K][4];
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[k][threadIdx.x >> 6] = c[k];
  __syncthreads();
  if (threadIdx.x < K) {
    const int t = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
    if (t) atomicAdd(out + threadIdx.x, (unsigned long long)t);
  }
}

// Element-wise passes over a whole Np x Np matrix (Np even) walk it as
// pairs of doubles on a fixed grid, so that each workgroup adds its counts
// with one atomic per counter (one workgroup per 256 entries left ~10^5
// atomics on the same two words, which serialised the pass).
constexpr int kElemGrid = 2048;

__global__ void __launch_bounds__(256) k_count_positive(const double* X, int64_t count, unsigned long long* out) {
  int c[1] = {0};
  const double2* X2 = (const double2*)X;
  for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < count / 2; q += (int64_t)gridDim.x * 256) {
    const double2 x = X2[q];
    c[0] += (x.x > 0.0) + (x.y > 0.0);
  }
  block_count<1>(c, out);
}

// X += I (the doubling's increment) in place; counts the positive entries of
// the new X into out[0] and the entries whose value changed into out[1].
__global__ void __launch_bounds__(256)
k_stein_accumulate(double* X, const double* I, int64_t count, unsigned long long* out) {
  int c[2] = {0, 0};
  double2* X2 = (double2*)X;
  const double2* I2 = (const double2*)I;
  for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < count / 2; q += (int64_t)gridDim.x * 256) {
    const double2 x = X2[q], d = I2[q];
    const double2 y = {x.x + d.x, x.y + d.y};
    c[0] += (y.x > 0.0) + (y.y > 0.0);
    c[1] += (y.x != x.x) + (y.y != x.y);
    X2[q] = y;
  }
  block_count<2>(c, out);
}

__global__ void __launch_bounds__(256)
k_f64_emit(const double* X, int Np, int n, uint8_t* S, int64_t lds, double* Xo, int64_t ldx) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
    const double x = X[(int64_t)i * Np + j];
    S[(int64_t)i * lds + j] = x > 0.0 ? 1 : 0;
    if (Xo) Xo[(int64_t)i * ldx + j] = x;
  }
}

// Doubling loop on buffers already initialised: X = Q, B, and C (= B^T when
// c_is_bt).  T, Bn (and Cn unless c_is_bt) are scratch.  On return *Xp points
// at the buffer holding X.
static hipError_t stein_doubling(int64_t Np, double* X, double* B, double* C, double* T, double* Bn, double* Cn,
                                 bool c_is_bt, bool want_values, int max_doublings, hipStream_t s,
                                 unsigned long long* d_counter, unsigned long long* h_counter, int64_t* positives,
                                 int32_t* doublings, bool* done_out, std::string* err) {
  const dim3 tgrid((unsigned)(Np / 32), (unsigned)(Np / 32));
  EPS_CK(hipMemsetAsync(d_counter, 0, sizeof(unsigned long long), s), "counter clear");
  hipLaunchKernelGGL(k_count_positive, dim3(kElemGrid), dim3(256), 0, s, (const double*)X, (int64_t)Np * Np, d_counter);
  EPS_CK(hipGetLastError(), "count");
  EPS_CK(hipMemcpyAsync(h_counter, d_counter, sizeof(unsigned long long), hipMemcpyDeviceToHost, s), "readback");
  EPS_CK(hipStreamSynchronize(s), "sync");
  int64_t prev = (int64_t)h_counter[0];
  int j = 0;
  bool done = false;
  while (!done && j < max_doublings) {
    // Bn = B B;  Cn = C C;  T = B X;  I = T C (into B's buffer, free once T
    // is formed);  X += I;  B <- Bn, C <- Cn (or B^T).
    GemmArgs g1{B, Np, B, Np, nullptr, 0, Bn, Np, (int)Np, (int)Np, (int)Np, 0, -1};
    EPS_CK(dgemm(g1, s), "B B");
    if (!c_is_bt) {
      GemmArgs g1c{C, Np, C, Np, nullptr, 0, Cn, Np, (int)Np, (int)Np, (int)Np, 0, -1};
      EPS_CK(dgemm(g1c, s), "C C");
    }
    GemmArgs g2{B, Np, X, Np, nullptr, 0, T, Np, (int)Np, (int)Np, (int)Np, 0, -1};
    EPS_CK(dgemm(g2, s), "B X");
    GemmArgs g3{T, Np, C, Np, nullptr, 0, B, Np, (int)Np, (int)Np, (int)Np, 0, -1};
    EPS_CK(dgemm(g3, s), "T C");
    EPS_CK(hipMemsetAsync(d_counter, 0, 2 * sizeof(unsigned long long), s), "counter clear");
    hipLaunchKernelGGL(k_stein_accumulate, dim3(kElemGrid), dim3(256), 0, s, X, (const double*)B, (int64_t)Np * Np,
                       d_counter);
    EPS_CK(hipGetLastError(), "accumulate");
    std::swap(B, Bn);
    if (c_is_bt) {
      hipLaunchKernelGGL(k_transpose_f64, tgrid, dim3(256), 0, s, (const double*)B, C, (int)Np);
      EPS_CK(hipGetLastError(), "transpose");
    } else {
      std::swap(C, Cn);
    }
    EPS_CK(hipMemcpyAsync(h_counter, d_counter, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
           "readback");
    EPS_CK(hipStreamSynchronize(s), "sync");
    ++j;
    const int64_t c = (int64_t)h_counter[0];
    done = c == prev && (!want_values || h_counter[1] == 0);
    prev = c;
  }
  *positives = prev;
  *doublings = j;
  *done_out = done;
  return hipSuccess;
}

hipError_t sg_eps_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* P, int64_t ldp, double eps,
                        uint8_t* S, int64_t lds, double* X_out, int64_t ldx, int max_doublings, hipStream_t s,
                        int32_t* doublings, int64_t* positives, unsigned long long* d_counter,
                        unsigned long long* h_counter, std::string* err) {
  const int64_t Np = eps_padded_size(n);
  const size_t mat = (size_t)Np * Np;
  EPS_CK(ensure(ws, budget_left, 5 * mat * sizeof(double), "same-generation epsilon solve", err), *err);
  double* X = (double*)ws->buf;
  double* A = X + mat;
  double* AT = A + mat;
  double* T = AT + mat;
  double* An = T + mat;
  const dim3 rows((unsigned)((Np + 255) / 256), (unsigned)Np);
  // X_0 = eps I, A_0 = sqrt(eps) P, C = A^T
  hipLaunchKernelGGL(k_f64_from_bytes, rows, dim3(256), 0, s, (const uint8_t*)nullptr, (int64_t)0, (int)n, (int)Np,
                     eps, 1, X);
  hipLaunchKernelGGL(k_f64_from_bytes, rows, dim3(256), 0, s, P, ldp, (int)n, (int)Np, sqrt(eps), 0, A);
  hipLaunchKernelGGL(k_transpose_f64, dim3((unsigned)(Np / 32), (unsigned)(Np / 32)), dim3(256), 0, s,
                     (const double*)A, AT, (int)Np);
  EPS_CK(hipGetLastError(), "init");
  bool done = false;
  EPS_CK(stein_doubling(Np, X, A, AT, T, An, nullptr, true, X_out != nullptr, max_doublings, s, d_counter, h_counter,
                        positives, doublings, &done, err),
         *err);
  hipLaunchKernelGGL(k_f64_emit, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, s, (const double*)X,
                     (int)Np, (int)n, S, lds, X_out, ldx);
  EPS_CK(hipGetLastError(), "threshold");
  EPS_CK(hipStreamSynchronize(s), "sync");
  return done ? hipSuccess : hipErrorNotReady;
}

hipError_t two_sided_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* Q, int64_t ldq,
                           const uint8_t* B, int64_t ldb, const uint8_t* C, int64_t ldc, double eps, uint8_t* R,
                           int64_t ldr, double* X_out, int64_t ldx, int8_t* R8, int64_t ld8,
                           unsigned long long* r8_count, int max_doublings, hipStream_t s, int32_t* doublings, unsigned long long* d_counter,
                           unsigned long long* h_counter, std::string* err) {
  const int64_t Np = eps_padded_size(n);
  const size_t mat = (size_t)Np * Np;
  EPS_CK(ensure(ws, budget_left, 6 * mat * sizeof(double), "two-sided solve", err), *err);
  double* X = (double*)ws->buf;
  double* Bd = X + mat;
  double* Cd = Bd + mat;
  double* T = Cd + mat;
  double* Bn = T + mat;
  double* Cn = Bn + mat;
  const dim3 rows((unsigned)((Np + 255) / 256), (unsigned)Np);
  // X = eps (Q + B X C): X_0 = eps Q, B_0 = sqrt(eps) B, C_0 = sqrt(eps) C
  const double se = sqrt(eps);
  hipLaunchKernelGGL(k_f64_from_bytes, rows, dim3(256), 0, s, Q, ldq, (int)n, (int)Np, eps, 0, X);
  hipLaunchKernelGGL(k_f64_from_bytes, rows, dim3(256), 0, s, B, ldb, (int)n, (int)Np, se, 0, Bd);
  hipLaunchKernelGGL(k_f64_from_bytes, rows, dim3(256), 0, s, C, ldc, (int)n, (int)Np, se, 0, Cd);
  EPS_CK(hipGetLastError(), "init");
  bool done = false;
  int64_t pos = 0;
  EPS_CK(stein_doubling(Np, X, Bd, Cd, T, Bn, Cn, false, X_out != nullptr, max_doublings, s, d_counter, h_counter,
                        &pos, doublings, &done, err),
         *err);
  if (R) {
    hipLaunchKernelGGL(k_f64_emit, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, s, (const double*)X,
                       (int)Np, (int)n, R, ldr, X_out, ldx);
    EPS_CK(hipGetLastError(), "threshold");
  }
  if (R8) {
    StackDesc d{};
    d.M = 1;
    d.Np = (int)Np;
    d.R[0] = R8;
    d.ldr = ld8;
    d.cnt = r8_count;
    hipLaunchKernelGGL(k_stack_emit, dim3((unsigned)((Np + 255) / 256), (unsigned)Np), dim3(256), 0, s, d,
                       (int64_t)0, (int64_t)Np, (const double*)X);
    EPS_CK(hipGetLastError(), "threshold");
  }
  EPS_CK(hipStreamSynchronize(s), "sync");
  return done ? hipSuccess : hipErrorNotReady;
}

#undef EPS_CK

}  // namespace dl
