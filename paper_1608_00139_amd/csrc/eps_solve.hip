// eps_solve.hip -- the epsilon form of Sec. 4 (Proposition 1, Theorem 1):
// X = (I - eps A)^-1 eps A in fp64, then R = [X > 0].
//
// Method: block Gaussian elimination without pivoting on the augmented matrix
// W = [ I - eps A | eps A ]  (Np x 2Np, row-major), block size NB = 128, with
// every diagonal block normalised to the identity:
//   for each block row k (rows K0 .. K0+NB):
//     Dinv  = W_kk^-1                      (Gauss-Jordan, one workgroup)
//     T     = Dinv * W[k, K0+NB : 2Np]     (fp64 MFMA product)
//     W[below, K0+NB : 2Np] -= W[below, k] * T   (trailing update, fp64 MFMA)
//     W[k, K0+NB : 2Np] = T
// leaving a block upper-triangular system with identity diagonal blocks,
// then back substitution, bottom block row first:
//     W[0 : K0, Np : 2Np] -= W[0 : K0, k] * W[k, Np : 2Np]
// after which the right half of W holds X.
//
// Why no pivoting: M = I - eps A has unit diagonal and off-diagonal entries
// <= 0 with eps * (row sum of A) < 1 (Lemma 1's eps bound), so M is a
// strictly diagonally dominant M-matrix; its Schur complements stay
// M-matrices, their inverses are entrywise >= 0, and every update above adds
// terms of one sign to the off-diagonal and right-hand-side entries.  Exact
// zeros therefore stay exactly zero and positive entries never cancel:
// thresholding at > 0 is exact except where a true value underflows fp64
// (it is at least eps^L for a shortest path of length L, by the footnote to
// Lemma 2).  Denormals are kept.
#include <math.h>

#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "eps_solve.h"

namespace dl {

constexpr int NB = 128;  // block size of the elimination

// ----------------------------------------------------------------- fp64 MFMA GEMM
// D = beta * C + alpha * A * B,  A: M x K, B: K x N, C/D: M x N, row-major.
// M, N multiples of 128, K multiple of 16.  D may alias C (same element
// read then written by the same lane); A and B must not overlap D.
struct GemmArgs {
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  const double* C; int64_t ldc;
  double* D; int64_t ldd;
  int M, N, K;
  double alpha;
  int beta;  // 0 or 1
};

// Output coordinate of accumulator element `item` of lane `lane` for
// v_mfma_f64_16x16x4f64 (gfx950), as measured on the device.
__device__ inline void f64_acc_coord(int lane, int item, int& r, int& c) {
  r = (lane >> 4) + 4 * item;
  c = lane & 15;
}

template <int BM, int BN, int BK>
__global__ void __launch_bounds__(256) k_dgemm(GemmArgs g) {
  constexpr int WM = BM / 2, WN = BN / 2;   // 2 x 2 waves
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int PAD = 2;
  __shared__ double As[BK][BM + PAD];
  __shared__ double Bs[BK][BN + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int tiles_n = g.N / BN;
  // column-major walk over tiles keeps one B column panel hot across rows
  const int tm = blockIdx.x % (g.M / BM), tn = blockIdx.x / (g.M / BM);
  (void)tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  v4d acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  constexpr int ACH = BM * BK / 2;   // 16-byte chunks of the A tile
  constexpr int BCH = BK * BN / 2;
  constexpr int AL = ACH / 256, BL = BCH / 256;
  static_assert(ACH % 256 == 0 && BCH % 256 == 0, "tile loads must divide evenly");
  double2 ra[AL], rb[BL];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AL; ++i) {
      const int q = tid + i * 256;
      const int row = q / (BK / 2), kk = (q % (BK / 2)) * 2;
      ra[i] = *(const double2*)(g.A + (int64_t)(m0 + row) * g.lda + k0 + kk);
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int q = tid + i * 256;
      const int k = q / (BN / 2), nn = (q % (BN / 2)) * 2;
      rb[i] = *(const double2*)(g.B + (int64_t)(k0 + k) * g.ldb + n0 + nn);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int i = 0; i < AL; ++i) {
      const int q = tid + i * 256;
      const int row = q / (BK / 2), kk = (q % (BK / 2)) * 2;
      As[kk][row] = ra[i].x;
      As[kk + 1][row] = ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int q = tid + i * 256;
      const int k = q / (BN / 2), nn = (q % (BN / 2)) * 2;
      *(double2*)&Bs[k][nn] = rb[i];
    }
  };

  const int g4 = lane >> 4, r16 = lane & 15;
  gload(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();  // previous stage fully consumed
    sstore();
    __syncthreads();
    if (k0 + BK < g.K) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = As[kk + g4][wm * WM + i * 16 + r16];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = Bs[kk + g4][wn * WN + j * 16 + r16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r, c;
        f64_acc_coord(lane, v, r, c);
        const int gr = m0 + wm * WM + i * 16 + r, gc = n0 + wn * WN + j * 16 + c;
        double x = g.alpha * acc[i][j][v];
        if (g.beta) x += g.C[(int64_t)gr * g.ldc + gc];
        g.D[(int64_t)gr * g.ldd + gc] = x;
      }
}

static hipError_t dgemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.M % 128 || g.N % 128 || g.K % 16) return hipErrorInvalidValue;
  const int grid = (g.M / 128) * (g.N / 128);
  hipLaunchKernelGGL((k_dgemm<128, 128, 16>), dim3(grid), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ----------------------------------------------------------------- diagonal block inverse
// In-place Gauss-Jordan inversion of the NB x NB block at W (ld), written to
// Dinv (ld NB).  1024 threads; thread t owns row t / 8 and the 16 columns
// (t % 8) + 8 m.  Step p broadcasts row p and column p through LDS (double
// buffered, one barrier per step):
//   row p:     a[p][j] /= a[p][p]  (j != p),   a[p][p] = 1 / a[p][p]
//   other i:   a[i][j] -= a[i][p] a[p][j] / a[p][p]  (j != p),
//              a[i][p]  = -a[i][p] / a[p][p]
__global__ void __launch_bounds__(1024) k_block_inverse(const double* W, int64_t ld, double* Dinv) {
  __shared__ double rowbuf[2][NB];
  __shared__ double colbuf[2][NB];
  const int t = threadIdx.x;
  const int i = t >> 3, j0 = t & 7;
  double a[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) a[m] = W[(int64_t)i * ld + j0 + 8 * m];
  for (int p = 0; p < NB; ++p) {
    const int b = p & 1;
    if (i == p) {
#pragma unroll
      for (int m = 0; m < 16; ++m) rowbuf[b][j0 + 8 * m] = a[m];
    }
    if (j0 == (p & 7)) {
#pragma unroll
      for (int m = 0; m < 16; ++m)
        if (m == (p >> 3)) colbuf[b][i] = a[m];
    }
    __syncthreads();
    const double inv = 1.0 / rowbuf[b][p];
    const double f = colbuf[b][i];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int j = j0 + 8 * m;
      if (i == p) {
        a[m] = (j == p) ? inv : a[m] * inv;
      } else if (j == p) {
        a[m] = -f * inv;
      } else {
        a[m] -= f * (rowbuf[b][j] * inv);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) Dinv[i * NB + j0 + 8 * m] = a[m];
}

// ----------------------------------------------------------------- setup / copy / emit
// W[i][j] = [i == j] - eps a_ij  and  W[i][Np + j] = eps a_ij, padded rows and
// columns carry the identity and zeros.
__global__ void __launch_bounds__(256)
k_eps_init(const uint8_t* A, int64_t lda, int n, int Np, double eps, double* W) {
  const int i = blockIdx.y;
  const int64_t ld = 2 * (int64_t)Np;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < Np; j += gridDim.x * 256) {
    const double a = (i < n && j < n && A[(int64_t)i * lda + j] != 0) ? 1.0 : 0.0;
    W[i * ld + j] = (i == j ? 1.0 : 0.0) - eps * a;
    W[i * ld + Np + j] = eps * a;
  }
}

__global__ void __launch_bounds__(256)
k_copy_rows(const double* src, int64_t lds, double* dst, int64_t ldd, int rows, int cols) {
  const int r = blockIdx.y;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < cols; c += gridDim.x * 256)
    dst[(int64_t)r * ldd + c] = src[(int64_t)r * lds + c];
  (void)rows;
}

__global__ void __launch_bounds__(256)
k_eps_emit(const double* W, int Np, int n, uint8_t* R, int64_t ldr, double* X, int64_t ldx) {
  const int i = blockIdx.y;
  const int64_t ld = 2 * (int64_t)Np;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
    const double x = W[i * ld + Np + j];
    R[(int64_t)i * ldr + j] = x > 0.0 ? 1 : 0;
    if (X) X[(int64_t)i * ldx + j] = x;
  }
}

// ----------------------------------------------------------------- driver
int64_t eps_padded_size(int64_t n) { return n <= 0 ? 0 : ((n + NB - 1) / NB) * NB; }

void eps_free(EpsWorkspace* ws) {
  if (ws->buf) (void)hipFree(ws->buf);
  ws->buf = nullptr;
  ws->size = 0;
}

hipError_t eps_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* A, int64_t lda,
                     double eps, uint8_t* R, int64_t ldr, double* X_out, int64_t ldx, hipStream_t s,
                     bool timing, double* trailing_ms, int64_t* trailing_launches, std::string* err) {
  *trailing_ms = 0.0;
  *trailing_launches = 0;
  const int64_t Np = eps_padded_size(n);
  const int64_t ldw = 2 * Np;
  const size_t wbytes = (size_t)Np * ldw * sizeof(double);
  const size_t dbytes = (size_t)NB * NB * sizeof(double);
  const size_t tbytes = (size_t)NB * ldw * sizeof(double);
  const size_t need = wbytes + dbytes + tbytes;
  if (need > ws->size) {
    if (budget_left && need > budget_left) {
      *err = "epsilon-solve workspace of " + std::to_string(need) + " bytes exceeds the budget";
      return hipErrorOutOfMemory;
    }
    eps_free(ws);
    hipError_t e = hipMalloc(&ws->buf, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ws->buf = nullptr;
      *err = "hipMalloc of " + std::to_string(need) + " bytes for the epsilon solve failed";
      return hipErrorOutOfMemory;
    }
    ws->size = need;
  }
  double* W = (double*)ws->buf;
  double* Dinv = W + (size_t)Np * ldw;
  double* T = Dinv + (size_t)NB * NB;
  hipError_t e;
#define EPS_CK(x, what)            \
  do {                             \
    e = (x);                       \
    if (e != hipSuccess) {         \
      *err = what;                 \
      return e;                    \
    }                              \
  } while (0)

  hipLaunchKernelGGL(k_eps_init, dim3((unsigned)((Np + 255) / 256), (unsigned)Np), dim3(256), 0, s, A, lda,
                     (int)n, (int)Np, eps, W);
  EPS_CK(hipGetLastError(), "epsilon init");

  std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
  const int nblk = (int)(Np / NB);
  for (int k = 0; k < nblk; ++k) {
    const int64_t K0 = (int64_t)k * NB;
    const int cols = (int)(ldw - K0 - NB);  // columns right of the diagonal block
    hipLaunchKernelGGL(k_block_inverse, dim3(1), dim3(1024), 0, s, W + K0 * ldw + K0, ldw, Dinv);
    EPS_CK(hipGetLastError(), "block inverse");
    GemmArgs rp{Dinv, NB, W + K0 * ldw + K0 + NB, ldw, nullptr, 0, T, ldw, NB, cols, NB, 1.0, 0};
    EPS_CK(dgemm(rp, s), "row panel product");
    const int below = (int)(Np - K0 - NB);
    if (below > 0) {
      GemmArgs tu{W + (K0 + NB) * ldw + K0, ldw, T, ldw, W + (K0 + NB) * ldw + K0 + NB, ldw,
                  W + (K0 + NB) * ldw + K0 + NB, ldw, below, cols, NB, -1.0, 1};
      hipEvent_t ea = nullptr, eb = nullptr;
      if (timing && hipEventCreate(&ea) == hipSuccess && hipEventCreate(&eb) == hipSuccess) {
        (void)hipEventRecord(ea, s);
      }
      EPS_CK(dgemm(tu, s), "trailing update");
      if (ea && eb) {
        (void)hipEventRecord(eb, s);
        evs.push_back({ea, eb});
      }
    }
    hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((cols + 255) / 256), NB), dim3(256), 0, s, T, ldw,
                       W + K0 * ldw + K0 + NB, ldw, NB, cols);
    EPS_CK(hipGetLastError(), "row panel copy");
  }
  for (int k = nblk - 1; k >= 1; --k) {
    const int64_t K0 = (int64_t)k * NB;
    GemmArgs bs{W + K0, ldw, W + K0 * ldw + Np, ldw, W + Np, ldw, W + Np, ldw, (int)K0, (int)Np, NB, -1.0, 1};
    EPS_CK(dgemm(bs, s), "back substitution");
  }
  hipLaunchKernelGGL(k_eps_emit, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, s, W, (int)Np,
                     (int)n, R, ldr, X_out, ldx);
  EPS_CK(hipGetLastError(), "threshold");
  EPS_CK(hipStreamSynchronize(s), "epsilon solve sync");
  for (auto& p : evs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, p.first, p.second) == hipSuccess) {
      *trailing_ms += t;
      *trailing_launches += 1;
    }
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
#undef EPS_CK
  return hipSuccess;
}

}  // namespace dl
