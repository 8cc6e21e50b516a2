// prog_kernels.hip -- elementwise kernels on int8 0/1 matrices (Np x Np,
// row-major, zero padded): disjunction of relations, complement for negated
// atoms (Sec. 8), transposed copies for converse atoms, the column-sum norm,
// the edge-list scatter that admits serving requests, the serving rounds'
// descriptor upload (which drops the products of finished requests), the
// fixpoint driver's read-back into pinned host memory, and the pseudo-random
// relation the tile autotuner times its candidates on.
#include "common.h"

namespace dl {

// out = op(a | b | I) on a 64 x 64 tile per workgroup (256 threads, 16 bytes
// each); `complement` turns the tile into [i < n, j < n] & !v.  Writes out
// and/or outT (the transpose, through LDS) and adds the tile's ones to *cnt.
__global__ void __launch_bounds__(256)
k_bytes_op(const int8_t* a, const int8_t* b, int ident, int complement, int n, int Np,
           int8_t* out, int8_t* outT, unsigned long long* cnt) {
  __shared__ uint8_t tile[64][64 + 16];
  const int bi = blockIdx.y, bj = blockIdx.x;
  const int tid = threadIdx.x;
  const int r = tid >> 2, c0 = (tid & 3) * 16;
  const int gi = bi * 64 + r, gj0 = bj * 64 + c0;
  const int64_t off = (int64_t)gi * Np + gj0;
  u32x4 v = {0u, 0u, 0u, 0u};
  if (a) v |= *(const u32x4*)(a + off);
  if (b) v |= *(const u32x4*)(b + off);
  if (ident && gi < n && gi >= gj0 && gi < gj0 + 16) {
    const int t = gi - gj0;
    v[t >> 2] |= 1u << (8 * (t & 3));
  }
  if (complement) {
    u32x4 m = {0u, 0u, 0u, 0u};
    if (gi < n) {
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (gj0 + t < n) m[t >> 2] |= 1u << (8 * (t & 3));
    }
    v = m & ~v;
  }
  if (out) *(u32x4*)(out + off) = v;
  int ones = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) ones += __popc(v[w]);
  if (outT) {
    *(u32x4*)&tile[r][c0] = v;
    __syncthreads();
    u32x4 t;
#pragma unroll
    for (int w = 0; w < 4; ++w)
      t[w] = (unsigned)tile[c0 + 4 * w][r] | ((unsigned)tile[c0 + 4 * w + 1][r] << 8) |
             ((unsigned)tile[c0 + 4 * w + 2][r] << 16) | ((unsigned)tile[c0 + 4 * w + 3][r] << 24);
    *(u32x4*)(outT + (int64_t)(bj * 64 + r) * Np + bi * 64 + c0) = t;
  }
  if (cnt) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ones += __shfl_xor(ones, o, 64);
    __shared__ int red[4];
    if ((tid & 63) == 0) red[tid >> 6] = ones;
    __syncthreads();
    if (tid == 0) {
      const int t = red[0] + red[1] + red[2] + red[3];
      if (t) atomicAdd(cnt, (unsigned long long)t);
    }
  }
}

hipError_t launch_bytes_op(const int8_t* a, const int8_t* b, int ident, int complement, int n, int Np, int8_t* out,
                           int8_t* outT, unsigned long long* cnt, hipStream_t s) {
  if (Np % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bytes_op, dim3(Np / 64, Np / 64), dim3(256), 0, s, a, b, ident, complement, n, Np, out, outT,
                     cnt);
  return hipGetLastError();
}

// Largest column sum: each thread walks one column (consecutive threads take
// consecutive columns, so every row read is coalesced).
__global__ void __launch_bounds__(256) k_col_max(const uint8_t* A, int64_t lda, int n, int* out_max) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  int s = 0;
  for (int i = 0; i < n; ++i) s += A[(int64_t)i * lda + j] != 0;
  atomicMax(out_max, s);
}

hipError_t launch_col_max(const uint8_t* A, int64_t lda, int n, int* out_max, hipStream_t s) {
  hipLaunchKernelGGL(k_col_max, dim3((n + 255) / 256), dim3(256), 0, s, A, lda, n, out_max);
  return hipGetLastError();
}

// Relation from an edge list: for each (i, j) with 0 <= i, j < n, set byte
// (i, j) of M and, when set, of M2 and byte (j, i) of MT (all Np x Np, zeroed
// beforehand).  Duplicate edges are counted once: the byte of M is set with
// an atomic OR on its 32-bit word, and only the edge that flips it counts.
// Edges outside [0, n) are skipped.
__global__ void __launch_bounds__(256)
k_scatter_edges(const int32_t* __restrict__ edges, int64_t m, int n, int Np, int8_t* M, int8_t* M2, int8_t* MT,
                unsigned long long* ones) {
  int c = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
    const int i = edges[2 * e], j = edges[2 * e + 1];
    if (i < 0 || j < 0 || i >= n || j >= n) continue;
    const int64_t off = (int64_t)i * Np + j;
    unsigned* w = (unsigned*)(M + (off & ~(int64_t)3));
    const unsigned bit = 1u << (8 * (off & 3));
    const unsigned old = atomicOr(w, bit);
    if (!(old & bit)) ++c;
    if (M2) M2[off] = 1;
    if (MT) MT[(int64_t)j * Np + i] = 1;
  }
  if (!ones) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = red[0] + red[1] + red[2] + red[3];
    if (t) atomicAdd(ones, (unsigned long long)t);
  }
}

hipError_t launch_scatter_edges(const int32_t* edges, int64_t m, int n, int Np, int8_t* M, int8_t* M2, int8_t* MT,
                                unsigned long long* ones, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t blocks = (m + 255) / 256;
  hipLaunchKernelGGL(k_scatter_edges, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, edges, m, n,
                     Np, M, M2, MT, ones);
  return hipGetLastError();
}

// ---- grouped admission of serving requests (two launches per round)
// Last request whose running total start(d) is <= x.
template <class F>
__device__ inline int find_req(int nreq, long long x, F start) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start(mid) <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Clear every request's region in 16-byte units; units inside the identity
// block get the diagonal bytes (i, i) for i < n; the thread that clears a
// request's first unit zeroes its counter.  The requests' first units are
// read into LDS once, so each unit's request is found by a search in LDS
// (not by a chain of dependent global loads), and the unit's row in the
// identity block by a 32-bit division (np^2 < 2^32).
__global__ void __launch_bounds__(256) k_admit_clear(const AdmitDesc* __restrict__ d, int nreq, long long total) {
  extern __shared__ long long s_first[];  // nreq entries
  for (int i = threadIdx.x; i < nreq; i += 256) s_first[i] = d[i].clear_start;
  __syncthreads();
  for (long long u = (long long)blockIdx.x * 256 + threadIdx.x; u < total; u += (long long)gridDim.x * 256) {
    const int q = find_req(nreq, u, [&](int i) { return s_first[i]; });
    const long long local = u - s_first[q];
    const AdmitDesc& a = d[q];
    u32x4 v = {0u, 0u, 0u, 0u};
    const long long ident = a.ident_off;
    if (ident >= 0) {
      const long long o = local * 16 - ident;
      const unsigned np = (unsigned)a.Np;
      if (o >= 0 && o < (long long)np * np) {
        const unsigned i = (unsigned)o / np, j0 = (unsigned)o - i * np;
        if ((int)i < a.n && i >= j0 && i < j0 + 16) {
          const int t = (int)(i - j0);
          v[t >> 2] |= 1u << (8 * (t & 3));
        }
      }
    }
    *(u32x4*)(a.base + local * 16) = v;
    if (local == 0 && a.ones) *a.ones = 0ull;
  }
}

// Scatter every request's edges (as k_scatter_edges).  A wave whose lanes all
// hold edges of one request adds its distinct-edge count with one atomic.
__global__ void __launch_bounds__(256) k_admit_scatter(const AdmitDesc* __restrict__ d, int nreq, long long total) {
  extern __shared__ long long s_first[];  // nreq entries: each request's first edge
  for (int i = threadIdx.x; i < nreq; i += 256) s_first[i] = d[i].edge_start;
  __syncthreads();
  for (long long e0 = (long long)blockIdx.x * 256; e0 < total; e0 += (long long)gridDim.x * 256) {
    const long long e = e0 + threadIdx.x;
    int q = -1, c = 0;
    if (e < total) {
      q = find_req(nreq, e, [&](int i) { return s_first[i]; });
      const AdmitDesc& a = d[q];
      const long long k = e - a.edge_start;
      const int i = a.edges[2 * k], j = a.edges[2 * k + 1];
      if (i >= 0 && j >= 0 && i < a.n && j < a.n) {
        const int64_t off = (int64_t)i * a.Np + j;
        unsigned* w = (unsigned*)(a.M + (off & ~(int64_t)3));
        const unsigned bit = 1u << (8 * (off & 3));
        if (!(atomicOr(w, bit) & bit)) c = 1;
        if (a.M2) a.M2[off] = 1;
        if (a.MT) a.MT[(int64_t)j * a.Np + i] = 1;
      }
    }
    const int q0 = __shfl(q, 0, 64);
    if (__all(q == q0)) {
      int t = c;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
      if ((threadIdx.x & 63) == 0 && t && q0 >= 0 && d[q0].ones) atomicAdd(d[q0].ones, (unsigned long long)t);
    } else if (c && d[q].ones) {
      atomicAdd(d[q].ones, 1ull);
    }
  }
}

hipError_t launch_admit(const AdmitDesc* d, int nreq, long long total_units, long long total_edges, hipStream_t s) {
  if (nreq <= 0) return hipSuccess;
  if (nreq > kRing) return hipErrorInvalidValue;  // the LDS copy of the requests' starts (32 KB at most)
  if (total_units > 0) {
    const long long blocks = (total_units + 255) / 256;
    hipLaunchKernelGGL(k_admit_clear, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256),
                       (size_t)nreq * sizeof(long long), s, d, nreq, total_units);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (total_edges > 0) {
    const long long blocks = (total_edges + 255) / 256;
    hipLaunchKernelGGL(k_admit_scatter, dim3((unsigned)(blocks < 2048 ? blocks : 2048)), dim3(256),
                       (size_t)nreq * sizeof(long long), s, d, nreq, total_edges);
    return hipGetLastError();
  }
  return hipSuccess;
}

// dst[i] = src[i] for i < n 8-byte words, one side a device mapping of
// coherent pinned host memory: the fixpoint driver's read-back of a slot's
// model sizes and convergence step, and the serving rounds' descriptor
// uploads and counter read-backs, as ordinary launches that follow the step
// launches without the gap a runtime copy leaves before it.
__global__ void __launch_bounds__(256) k_publish(const unsigned long long* __restrict__ src, unsigned long long* dst,
                                                 int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) dst[i] = src[i];
}

hipError_t launch_publish(const unsigned long long* src, unsigned long long* dst, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_publish, dim3(blocks < 64 ? blocks : 64), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// A serving round's descriptor upload (in place of a k_publish of them),
// compacting its tile lists: a product issued before the previous round's
// model sizes were read back, of a request that finished in that round
// (*chk == chk_val), gets no tiles, and the other products' tiles are
// renumbered without gaps, so that the persistent launches deal only live
// tiles and stay balanced.  A descriptor without tiles keeps its place: its
// tile_start equals the next one's, and the grouped kernels' search (the last
// request whose first tile is <= the item) passes over it.  One workgroup;
// thread q handles descriptors [q c, q c + c), c = ceil(all / 1024) <= 4.
constexpr int kUploadThreads = 1024;
constexpr int kUploadPerThread = (kMaxGroupRequests + kUploadThreads - 1) / kUploadThreads;

__global__ void __launch_bounds__(kUploadThreads)
k_group_upload(const GroupDesc* __restrict__ src, GroupDesc* __restrict__ dst, GroupLists L, int* __restrict__ totals) {
  __shared__ int s_wave[kUploadThreads / 64];
  __shared__ int s_base[4];
  const int nall = L.begin[3];
  const int q = threadIdx.x, lane = q & 63, w = q >> 6;
  const int c = (nall + kUploadThreads - 1) / kUploadThreads;
  const int i0 = min(q * c, nall), i1 = min(i0 + c, nall);
  auto segment = [&](int i) { return i < L.begin[1] ? 0 : (i < L.begin[2] ? 1 : 2); };
  int live[kUploadPerThread];
  int sum = 0;
#pragma unroll
  for (int j = 0; j < kUploadPerThread; ++j) {
    const int i = i0 + j;
    live[j] = 0;
    if (i < i1) {
      const GroupDesc g = src[i];
      const int side = g.Np / L.tile[segment(i)];
      const int tiles = g.sym ? side * (side + 1) / 2 : side * side;
      live[j] = (g.chk != nullptr && *g.chk == g.chk_val) ? 0 : tiles;
      dst[i] = g;  // tile_start is rewritten below (same thread, same address: in order)
      sum += live[j];
    }
  }
  // exclusive prefix of the per-thread sums: a scan in each wave, then the
  // totals of the waves before
  int incl = sum;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) s_wave[w] = incl;
  __syncthreads();
  int before = 0, total = 0;
  for (int x = 0; x < kUploadThreads / 64; ++x) {
    const int v = s_wave[x];
    before += x < w ? v : 0;
    total += v;
  }
  const int excl = before + incl - sum;
  // the prefix at each segment's first descriptor, from the thread holding it
  for (int k = 0; k < 4; ++k) {
    const int first = L.begin[k];
    if (first >= nall) {
      if (q == 0) s_base[k] = total;
    } else if (first >= i0 && first < i1) {
      int v = excl;
#pragma unroll
      for (int j = 0; j < kUploadPerThread; ++j) v += (i0 + j < first) ? live[j] : 0;
      s_base[k] = v;
    }
  }
  __syncthreads();
  int run = excl;
#pragma unroll
  for (int j = 0; j < kUploadPerThread; ++j) {
    const int i = i0 + j;
    if (i < i1) {
      dst[i].tile_start = run - s_base[segment(i)];
      run += live[j];
    }
  }
  if (q < 3) totals[q] = s_base[q + 1] - s_base[q];
}

hipError_t launch_group_upload(const GroupDesc* src, GroupDesc* dst, const GroupLists& L, int* totals, hipStream_t s) {
  const int nall = L.begin[3];
  if (nall <= 0) return hipSuccess;
  if (nall > kMaxGroupRequests || L.begin[0] != 0 || L.begin[1] < 0 || L.begin[1] > L.begin[2] ||
      L.begin[2] > L.begin[3] || !src || !dst || !totals)
    return hipErrorInvalidValue;
  for (int k = 0; k < 3; ++k)
    if (L.tile[k] != 64 && L.tile[k] != 128 && L.tile[k] != 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_group_upload, dim3(1), dim3(kUploadThreads), 0, s, src, dst, L, totals);
  return hipGetLastError();
}

// M[i][j] = a pseudo-random bit (density 1/2) for i, j < n, 0 in the padding
// up to Np; bits from the "lowbias32" integer hash (C. Wellons) of the
// element index mixed with the seed.
__global__ void __launch_bounds__(256) k_hash_bool(uint8_t* M, int64_t ld, int n, int Np, unsigned seed) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)Np * Np) return;
  const int i = (int)(idx / Np), j = (int)(idx % Np);
  unsigned x = (unsigned)idx ^ (seed * 0x9e3779b9u);
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  M[(int64_t)i * ld + j] = (i < n && j < n) ? (uint8_t)((x >> 7) & 1u) : (uint8_t)0;
}

hipError_t launch_hash_bool(uint8_t* M, int64_t ld, int n, int Np, unsigned seed, hipStream_t s) {
  const int64_t total = (int64_t)Np * Np;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_bool, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, M, ld, n, Np, seed);
  return hipGetLastError();
}

}  // namespace dl
