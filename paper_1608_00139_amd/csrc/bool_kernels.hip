// bool_kernels.hip -- boolean fixpoint steps on gfx950 matrix cores.
//
// Every step of the three fixpoints is one "NT" product with a fused
// threshold:   out(i, j) = [ add(i, j) + sum_k X(i, k) Y(j, k)  !=  0 ].
// Both operands are row-major with K contiguous, the layout the MFMA
// operand registers want.  The fixpoint driver launches the products of the
// paper as follows (no addend: each closure step adds the previous iterate,
// which leaves the iterates unchanged, folded into the right operand as an
// identity):
//   closure, plain   R' = min1(A + A R)     run transposed: S = R^T,
//                    S' = [S (A + I)^T]     X = S, Y = A + I (written once
//                                           at ingest)
//   closure, squared R' = min1(A + R R)     X = R, Y = R^T + I; the epilogue
//                    R' = [R (R + I)]       also writes R'^T + I, the next
//                                           step's Y (outT_ident)
//   same generation  T  = [P S]             X = P, Y = S (S is symmetric)
//                    S' = [I + T P^T]       X = T, Y = P, add = identity
// Layered programs still pass an addend (their running sums).
// min1 on the non-negative integer counts is the test "!= 0" (Sec. 2, 3).
//
// Operands hold exactly 0 or 1 in the chosen precision (int8, fp32, bf16,
// fp8 e4m3 or fp4 e2m1), so every product is exact: int32 accumulation, or
// fp32 accumulation of counts below 2^24.
//
// Kernel structure (k_nt_step): one workgroup computes a BM x BN output
// tile, staging BK-byte slices of its X and Y row panels through LDS with
// double buffering.  LDS holds each slice as 16-byte chunks ordered
// [chunk][row][16 B], so the 16 lanes that read one MFMA operand chunk read
// 256 contiguous bytes (no bank conflicts).  The epilogue stages the 0/1
// tile through LDS, ORs the addend with 16-byte loads, stores coalesced rows
// (and, for squaring, the transposed tile), and counts the ones of the tile
// with a wave reduction and a single atomic per workgroup.  The large-tile
// kernel (k_nt_dma, below) fetches its slices straight into LDS and keeps
// the tile in registers until the stores.  A launch first checks the
// device-side convergence state and returns at once if the fixpoint was
// already reached, so chunks of steps can be enqueued ahead.
#include "common.h"

namespace dl {

// ----------------------------------------------------------------- operand policies
// FR = rows (and columns) of one MFMA fragment; the 64 lanes form 64 / FR
// groups along K, lane l supplying row l % FR of its group's K range.
// CPL = 16-byte chunks per lane per MFMA.  A and B use the same K
// assignment, so the instruction's internal K order does not matter.
// coord() gives the output row/column of accumulator item i of a lane
// (layouts checked on the device).

// 16x16 output tile: item i of lane l is row 4 (l / 16) + i, column l % 16
__device__ inline void coord16(int lane, int i, int& r, int& c) {
  r = 4 * (lane >> 4) + i;
  c = lane & 15;
}

struct OpI8 {
  static constexpr int kPrec = P_I8;
  static constexpr int FR = 16, CPL = 1, NI = 4;
  __device__ static void coord(int lane, int i, int& r, int& c) { coord16(lane, i, r, c); }
  typedef v4i Acc;
  __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
  __device__ static Acc mma(const u32x4* a, const u32x4* b, Acc c) {
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(v4i, a[0]),
                                                 __builtin_bit_cast(v4i, b[0]), c, 0, 0, 0);
  }
  __device__ static bool nz(const Acc& c, int i) { return c[i] != 0; }
};

// v_mfma_i32_32x32x32_i8: item i of lane l is row 8 (i / 4) + 4 (l / 32) + i % 4,
// column l % 32
struct OpI8x32 {
  static constexpr int kPrec = P_I8;
  static constexpr int FR = 32, CPL = 1, NI = 16;
  __device__ static void coord(int lane, int i, int& r, int& c) {
    r = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    c = lane & 31;
  }
  typedef v16i Acc;
  __device__ static Acc zero() { return Acc{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}; }
  __device__ static Acc mma(const u32x4* a, const u32x4* b, Acc c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(v4i, a[0]),
                                                 __builtin_bit_cast(v4i, b[0]), c, 0, 0, 0);
  }
  __device__ static bool nz(const Acc& c, int i) { return c[i] != 0; }
};

struct OpF32 {
  static constexpr int kPrec = P_F32;
  static constexpr int FR = 16, CPL = 1, NI = 4;
  __device__ static void coord(int lane, int i, int& r, int& c) { coord16(lane, i, r, c); }
  typedef v4f Acc;
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static Acc mma(const u32x4* a, const u32x4* b, Acc c) {
    // one chunk = 4 consecutive k; four K=4 instructions, lane group g
    // supplies k = 4*chunk(g) + j in instruction j
    // bit-cast whole vectors: a scalar bit-cast of one element of an
    // unsigned ext-vector is miscompiled by this clang (it yields element 0)
    const v4f x = __builtin_bit_cast(v4f, a[0]), y = __builtin_bit_cast(v4f, b[0]);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, y.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, y.w, c, 0, 0, 0);
    return c;
  }
  __device__ static bool nz(const Acc& c, int i) { return c[i] != 0.f; }
};

struct OpBF16 {
  static constexpr int kPrec = P_BF16;
  static constexpr int FR = 16, CPL = 1, NI = 4;
  __device__ static void coord(int lane, int i, int& r, int& c) { coord16(lane, i, r, c); }
  typedef v4f Acc;
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static Acc mma(const u32x4* a, const u32x4* b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[0]),
                                                   __builtin_bit_cast(v8bf, b[0]), c, 0, 0, 0);
  }
  __device__ static bool nz(const Acc& c, int i) { return c[i] != 0.f; }
};

struct OpFP8 {
  static constexpr int kPrec = P_FP8;
  static constexpr int FR = 16, CPL = 2, NI = 4;
  __device__ static void coord(int lane, int i, int& r, int& c) { coord16(lane, i, r, c); }
  typedef v4f Acc;
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static Acc mma(const u32x4* a, const u32x4* b, Acc c) {
    v8i av, bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) { av[j] = a[0][j]; av[4 + j] = a[1][j]; bv[j] = b[0][j]; bv[4 + j] = b[1][j]; }
    // formats 0/0 = fp8 e4m3 for both operands; E8M0 scale 127 = 2^0
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
  }
  __device__ static bool nz(const Acc& c, int i) { return c[i] != 0.f; }
};

// fp4 e2m1 operands: 32 elements (16 bytes) per lane, K = 128 per instruction;
// 1.0 is the code 0x2.  The instruction reads the low four operand dwords.
struct OpFP4 {
  static constexpr int kPrec = P_FP4;
  static constexpr int FR = 16, CPL = 1, NI = 4;
  __device__ static void coord(int lane, int i, int& r, int& c) { coord16(lane, i, r, c); }
  typedef v4f Acc;
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static Acc mma(const u32x4* a, const u32x4* b, Acc c) {
    v8i av = {0, 0, 0, 0, 0, 0, 0, 0}, bv = {0, 0, 0, 0, 0, 0, 0, 0};
    const v4i x = __builtin_bit_cast(v4i, a[0]), y = __builtin_bit_cast(v4i, b[0]);
    av.lo = x;
    bv.lo = y;
    // formats 4/4 = fp4 e2m1 for both operands; E8M0 scale 127 = 2^0
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 4, 4, 0, 127, 0, 127);
  }
  __device__ static bool nz(const Acc& c, int i) { return c[i] != 0.f; }
};

// Store 16 boolean bytes (each 0 or 1) as 16 operand elements.
template <int PREC>
__device__ inline void store_bool16(uint8_t* dst, u32x4 b) {
  if constexpr (PREC == P_I8) {
    *(u32x4*)dst = b;
  } else if constexpr (PREC == P_FP4) {
    // two elements per byte: element 2t -> low nibble, 2t + 1 -> high nibble
    unsigned w2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const unsigned x = b[2 * h], y = b[2 * h + 1];
      const unsigned lo = ((x & 1u) << 1) | (((x >> 8) & 1u) << 5) | (((x >> 16) & 1u) << 9) | (((x >> 24) & 1u) << 13);
      const unsigned hi = ((y & 1u) << 1) | (((y >> 8) & 1u) << 5) | (((y >> 16) & 1u) << 9) | (((y >> 24) & 1u) << 13);
      w2[h] = lo | (hi << 16);
    }
    *(uint2*)dst = make_uint2(w2[0], w2[1]);
  } else if constexpr (PREC == P_FP8) {
    *(u32x4*)dst = b * 0x38u;  // bytes are 0/1: multiply puts 0x38 (1.0 in e4m3) in each set byte
  } else if constexpr (PREC == P_BF16) {
    u32x4 lo, hi;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      unsigned x = b[w];
      lo[2 * w] = ((x & 1u) ? 0x3F80u : 0u) | (((x >> 8) & 1u) ? 0x3F800000u : 0u);
      lo[2 * w + 1] = (((x >> 16) & 1u) ? 0x3F80u : 0u) | (((x >> 24) & 1u) ? 0x3F800000u : 0u);
      unsigned y = b[2 + w];
      hi[2 * w] = ((y & 1u) ? 0x3F80u : 0u) | (((y >> 8) & 1u) ? 0x3F800000u : 0u);
      hi[2 * w + 1] = (((y >> 16) & 1u) ? 0x3F80u : 0u) | (((y >> 24) & 1u) ? 0x3F800000u : 0u);
    }
    ((u32x4*)dst)[0] = lo;
    ((u32x4*)dst)[1] = hi;
  } else {  // F32
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      unsigned x = b[w];
      u32x4 v;
      v[0] = (x & 1u) ? 0x3F800000u : 0u;
      v[1] = ((x >> 8) & 1u) ? 0x3F800000u : 0u;
      v[2] = ((x >> 16) & 1u) ? 0x3F800000u : 0u;
      v[3] = ((x >> 24) & 1u) ? 0x3F800000u : 0u;
      ((u32x4*)dst)[w] = v;
    }
  }
}

// Nonzero test of one operand element, returned as 0/1.
template <int PREC>
__device__ inline unsigned elem_nz(const uint8_t* p, int64_t idx) {
  if constexpr (PREC == P_F32) return ((const unsigned*)p)[idx] != 0u ? 1u : 0u;
  else if constexpr (PREC == P_FP4) return ((p[idx >> 1] >> (4 * (idx & 1))) & 15u) != 0 ? 1u : 0u;
  else if constexpr (PREC == P_BF16) return ((const unsigned short*)p)[idx] != 0 ? 1u : 0u;
  else return p[idx] != 0 ? 1u : 0u;
}

// The 16 consecutive elements of precision PREC at base (aligned to 16
// elements) as 0/1 bytes, any nonzero element being true.
template <int PREC>
__device__ inline u32x4 bool16_of(const uint8_t* base) {
  u32x4 v = {0u, 0u, 0u, 0u};
  if constexpr (PREC == P_FP8 || PREC == P_I8) {
    u32x4 x = *(const u32x4*)base;  // fold each byte's bits into its bit 0
    x |= x >> 4;
    x |= x >> 2;
    x |= x >> 1;
    v = x & 0x01010101u;
  } else if constexpr (PREC == P_BF16) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const u32x4 w = ((const u32x4*)base)[h];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = 8 * h + 2 * j;  // elements e (low half) and e + 1 (high half)
        v[e >> 2] |= ((w[j] & 0xffffu) != 0u ? 1u : 0u) << (8 * (e & 3));
        v[(e + 1) >> 2] |= ((w[j] >> 16) != 0u ? 1u : 0u) << (8 * ((e + 1) & 3));
      }
    }
  } else if constexpr (PREC == P_F32) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const u32x4 w = ((const u32x4*)base)[h];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[h] |= (w[j] != 0u ? 1u : 0u) << (8 * j);
    }
  } else {  // fp4: element e is nibble e of the 8 bytes (low nibble first)
    const uint2 x = *(const uint2*)base;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const unsigned word = e < 8 ? x.x : x.y;
      v[e >> 2] |= (((word >> (4 * (e & 7))) & 15u) != 0u ? 1u : 0u) << (8 * (e & 3));
    }
  }
  return v;
}

// The 16 addend flags of row gr, columns gc .. gc + 15 (gc a multiple of 16)
// as 0/1 bytes: from an int8 0/1 addend, or (p.add_op) from an addend in the
// operand precision PREC, any nonzero element being true.
template <int PREC>
__device__ inline u32x4 load_add16(const NTParams& p, int gr, int gc) {
  if (PREC == P_I8 || !p.add_op) return *(const u32x4*)(p.add + (int64_t)gr * p.Np + gc);
  return bool16_of<PREC>((const uint8_t*)p.add + ((int64_t)gr * p.ld + gc) * elem_nibbles(PREC) / 2);
}

__device__ inline int popc16(u32x4 v) {
  return __builtin_popcount(v[0]) + __builtin_popcount(v[1]) + __builtin_popcount(v[2]) +
         __builtin_popcount(v[3]);
}

// v | the identity bit of its segment: row gr, columns gc .. gc + 15 hold
// the diagonal element (gr, gr) when gc <= gr < gc + 16 and gr < n.
__device__ inline u32x4 with_diag(u32x4 v, int gr, int gc, int n) {
  if (gr >= gc && gr < gc + 16 && gr < n) {
    const int b = gr - gc;
    v[b >> 2] |= 1u << (8 * (b & 3));
  }
  return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block index -> logical index.  The hardware deals workgroups round-robin
// over the 8 XCDs (block b on XCD b % 8); the blocks of XCD x get the
// contiguous run of logical indices [x q + min(x, r), ...), q = nblocks / 8,
// r = nblocks % 8 (a bijection on [0, nblocks) for any nblocks).
__device__ inline int xcd_logical(int b, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int x = b & 7, local = b >> 3;
  return x * q + (x < r ? x : r) + local;
}

// Block index -> output tile: each XCD takes a contiguous run of logical
// tiles, walked in groups of GM tile rows so that the workgroups resident on
// one XCD share row and column panels in its L2.
__device__ inline void tile_coords(int b, int nblocks, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int logical = xcd_logical(b, nblocks);
  constexpr int GM = 8;
  const int per_group = GM * tiles_n;
  const int group = logical / per_group;
  const int first_m = group * GM;
  const int gm = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
  const int in = logical - group * per_group;
  tm = first_m + in % gm;
  tn = in / gm;
}

// Early exit shared by every step launch: returns true if this launch has
// nothing to do because the fixpoint was reached before step p.step.
__device__ inline bool step_is_done(const NTParams& p) {
  if (!p.conv) return false;
  const int c = *(volatile const int*)p.conv;
  if (c < p.step) return true;
  if (p.check && p.step >= 2) {
    const unsigned long long a = *(volatile const unsigned long long*)(p.ones + ((p.step - 1) % kRing));
    const unsigned long long b = *(volatile const unsigned long long*)(p.ones + ((p.step - 2) % kRing));
    if (a == b) {
      if (threadIdx.x == 0) atomicMin(p.conv, p.step - 1);
      return true;
    }
  }
  return false;
}

// LDS row swizzle: the 16-byte chunk c of row r of a staged slice is stored
// at unit  c * rows + (r ^ swz(c)).  Lanes that store one global row (its KC
// chunks) then land in different banks, and the lanes that read one MFMA
// operand (consecutive rows of one chunk) still read a permutation of one
// aligned 8-row block.  swz < 8 keeps every row inside its aligned block.
template <int SWZ>
__device__ __host__ constexpr int swz(int c) {
  return SWZ ? ((c * SWZ) & 7) : 0;
}

template <int BM, int BN, int WM, int WN, int KB, class Op, int SWZ, int PREF = 1>
struct NTKernel {
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NWAVES = WAVES_M * WAVES_N;
  static constexpr int NT = NWAVES * 64;
  static constexpr int KC = KB / 16;                 // chunks per row per stage
  static constexpr int FR = Op::FR;
  static constexpr int GROUPS = 64 / FR;             // lane groups along K
  static constexpr int FM = WM / FR, FN = WN / FR;   // fragments per wave
  static constexpr int CPL = Op::CPL;
  static constexpr int KSTEP_CHUNKS = GROUPS * CPL;  // chunks consumed by one MFMA k-step
  static constexpr int KSTEPS = KC / KSTEP_CHUNKS;
  static constexpr int STAGE_CHUNKS = (BM + BN) * KC;
  static constexpr int LOADS = STAGE_CHUNKS / NT;
  static constexpr int EPAD = 16;
  static constexpr int EST = BN + EPAD;              // epilogue LDS row stride (bytes)
  static constexpr size_t OPER_BYTES = 2ull * STAGE_CHUNKS * 16;
  static constexpr size_t EPI_BYTES = (size_t)BM * EST;
  static constexpr size_t LDS_BYTES = OPER_BYTES > EPI_BYTES ? OPER_BYTES : EPI_BYTES;
  static constexpr int NIB = elem_nibbles(Op::kPrec);  // 4-bit units per element
  static_assert(KC % KSTEP_CHUNKS == 0, "stage must hold whole MFMA k-steps");
  static_assert(STAGE_CHUNKS % NT == 0, "loads must divide evenly");
  static_assert((BM * BN / 16) % NT == 0, "epilogue segments must divide evenly");
  static_assert(WM % FR == 0 && WN % FR == 0, "wave tile must hold whole fragments");
};

// One BM x BN output tile at (row0, col0) of out = [add + X Y^T != 0];
// its number of ones is added to *cnt_dst when cnt_dst is not null.  The
// whole workgroup must call it (it synchronises through LDS).
template <int BM, int BN, int WM, int WN, int KB, class Op, int SWZ, int PREF>
__device__ __forceinline__ void nt_tile(const NTParams& p, int row0, int col0,
                                        unsigned long long* cnt_dst, uint8_t* smem, int tid) {
  typedef NTKernel<BM, BN, WM, WN, KB, Op, SWZ, PREF> K;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / K::WAVES_N, wn = wave % K::WAVES_N;
  const int64_t ldb = p.ld * K::NIB / 2;  // row pitch in bytes
  const uint8_t* Xg = (const uint8_t*)p.X + (int64_t)row0 * ldb;
  const uint8_t* Yg = (const uint8_t*)p.Y + (int64_t)col0 * ldb;
  const int nk = (int)(ldb / KB);

  u32x4* lds = (u32x4*)smem;
  // chunk q of a stage: rows [0, BM) of X then rows [0, BN) of Y; the KC
  // chunks of one row are adjacent in global memory and in q
  auto gload = [&](u32x4 (&regs)[K::LOADS], int kt) {
#pragma unroll
    for (int i = 0; i < K::LOADS; ++i) {
      const int q = tid + i * K::NT;
      const int row = q / K::KC, c = q % K::KC;
      const uint8_t* src = (row < BM) ? (Xg + (int64_t)row * ldb) : (Yg + (int64_t)(row - BM) * ldb);
      regs[i] = *(const u32x4*)(src + (int64_t)kt * KB + c * 16);
    }
  };
  auto sstore = [&](const u32x4 (&regs)[K::LOADS], int buf) {
    u32x4* base = lds + buf * K::STAGE_CHUNKS;
#pragma unroll
    for (int i = 0; i < K::LOADS; ++i) {
      const int q = tid + i * K::NT;
      const int row = q / K::KC, c = q % K::KC;
      // X region: [KC][BM]; Y region after it: [KC][BN]
      const int off = (row < BM) ? (c * BM + (row ^ swz<SWZ>(c)))
                                 : (BM * K::KC + c * BN + ((row - BM) ^ swz<SWZ>(c)));
      base[off] = regs[i];
    }
  };

  typename Op::Acc acc[K::FM][K::FN];
#pragma unroll
  for (int i = 0; i < K::FM; ++i)
#pragma unroll
    for (int j = 0; j < K::FN; ++j) acc[i][j] = Op::zero();

  const int g = lane / K::FR, rf = lane % K::FR;
  auto compute = [&](int buf) {
    const u32x4* xs = lds + buf * K::STAGE_CHUNKS;
    const u32x4* ys = xs + BM * K::KC;
#pragma unroll
    for (int ks = 0; ks < K::KSTEPS; ++ks) {
      u32x4 af[K::FM][K::CPL], bf[K::FN][K::CPL];
#pragma unroll
      for (int i = 0; i < K::FM; ++i)
#pragma unroll
        for (int c = 0; c < K::CPL; ++c) {
          const int ch = ks * K::KSTEP_CHUNKS + g * K::CPL + c;
          af[i][c] = xs[ch * BM + ((wm * WM + i * K::FR + rf) ^ swz<SWZ>(ch))];
        }
#pragma unroll
      for (int j = 0; j < K::FN; ++j)
#pragma unroll
        for (int c = 0; c < K::CPL; ++c) {
          const int ch = ks * K::KSTEP_CHUNKS + g * K::CPL + c;
          bf[j][c] = ys[ch * BN + ((wn * WN + j * K::FR + rf) ^ swz<SWZ>(ch))];
        }
#pragma unroll
      for (int i = 0; i < K::FM; ++i)
#pragma unroll
        for (int j = 0; j < K::FN; ++j) acc[i][j] = Op::mma(af[i], bf[j], acc[i][j]);
    }
  };

  if constexpr (PREF == 1) {
    // one slice in flight: load k+1 into registers while computing k
    u32x4 ra[K::LOADS];
    gload(ra, 0);
    sstore(ra, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) gload(ra, kt + 1);
      compute(kt & 1);
      if (kt + 1 < nk) sstore(ra, (kt + 1) & 1);
      __syncthreads();
    }
  } else {
    // two slices in flight: the loads of slice k+1 had a whole compute phase
    // to land before they are stored to LDS at the end of iteration k
    u32x4 ra[K::LOADS], rb[K::LOADS];
    gload(ra, 0);
    if (nk > 1) gload(rb, 1);
    sstore(ra, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
      // even iteration: rb holds slice kt+1, ra is free
      if (kt + 2 < nk) gload(ra, kt + 2);
      compute(0);
      if (kt + 1 < nk) sstore(rb, 1);
      __syncthreads();
      if (kt + 1 >= nk) break;
      // odd iteration: ra holds slice kt+2, rb is free
      if (kt + 3 < nk) gload(rb, kt + 3);
      compute(1);
      if (kt + 2 < nk) sstore(ra, 0);
      __syncthreads();
    }
  }

  // ---- epilogue: 0/1 tile in LDS, [BM][EST] bytes
  constexpr int SEG_PER_ROW = BN / 16;
  constexpr int SEGS = BM * SEG_PER_ROW / K::NT;
  // int8 addend segments of this thread (segment i: tile row q / SEG_PER_ROW,
  // 16-byte column q % SEG_PER_ROW, q = tid + i NT), all requested before
  // the first is needed, so the tile waits on one memory round trip (wider
  // operand-precision addends are read per segment: held together they
  // would cost occupancy)
  constexpr bool BATCH = Op::kPrec == P_I8;
  u32x4 addv[SEGS];
#pragma unroll
  for (int i = 0; i < SEGS; ++i) {
    const int q = tid + i * K::NT;
    addv[i] = u32x4{0u, 0u, 0u, 0u};
    if (BATCH && p.add) addv[i] = load_add16<Op::kPrec>(p, row0 + q / SEG_PER_ROW, col0 + (q % SEG_PER_ROW) * 16);
  }
  uint8_t* et = smem;
#pragma unroll
  for (int i = 0; i < K::FM; ++i)
#pragma unroll
    for (int j = 0; j < K::FN; ++j)
#pragma unroll
      for (int v = 0; v < Op::NI; ++v) {
        int r, c;
        Op::coord(lane, v, r, c);
        et[(wm * WM + i * K::FR + r) * K::EST + wn * WN + j * K::FR + c] = Op::nz(acc[i][j], v) ? 1 : 0;
      }
  __syncthreads();

  int cnt = 0;
  uint8_t* outb = (uint8_t*)p.out;
#pragma unroll
  for (int i = 0; i < SEGS; ++i) {
    const int q = tid + i * K::NT;
    const int r = q / SEG_PER_ROW, cs = q % SEG_PER_ROW;
    u32x4 v = *(const u32x4*)(et + r * K::EST + cs * 16);
    const int gr = row0 + r, gc = col0 + cs * 16;
    if (BATCH) v |= addv[i];
    else if (p.add) v |= load_add16<Op::kPrec>(p, gr, gc);
    if (p.add_identity) v = with_diag(v, gr, gc, p.n_valid);
    cnt += popc16(v);
    store_bool16<Op::kPrec>(outb + ((int64_t)gr * p.ld + gc) * K::NIB / 2, v);
    if (p.outT) *(u32x4*)(et + r * K::EST + cs * 16) = p.outT_ident ? with_diag(v, gr, gc, p.n_valid) : v;
  }

  if (p.outT) {
    __syncthreads();
    constexpr int SEG_PER_COL = BM / 16;
    constexpr int TSEGS = BN * SEG_PER_COL / K::NT;
    uint8_t* outt = (uint8_t*)p.outT;
#pragma unroll 2
    for (int i = 0; i < TSEGS; ++i) {
      // consecutive lanes take consecutive columns of the same 16 rows, so
      // each byte read of a wave touches one 64-byte run of one LDS row
      const int q = tid + i * K::NT;
      const int c = q % BN, rs = q / BN;
      u32x4 v;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint8_t* e = et + (rs * 16 + 4 * w) * K::EST + c;
        v[w] = (unsigned)e[0] | ((unsigned)e[K::EST] << 8) | ((unsigned)e[2 * K::EST] << 16) |
               ((unsigned)e[3 * K::EST] << 24);
      }
      store_bool16<Op::kPrec>(outt + ((int64_t)(col0 + c) * p.ld + row0 + rs * 16) * K::NIB / 2, v);
    }
  }

  if (cnt_dst) {
    __shared__ int red[K::NWAVES];
    cnt = wave_sum(cnt);
    if (lane == 0) red[wave] = cnt;
    __syncthreads();
    if (tid == 0) {
      unsigned long long t = 0;
#pragma unroll
      for (int w = 0; w < K::NWAVES; ++w) t += (unsigned long long)red[w];
      // count 2: a tile of a symmetric product stands for its mirror image too
      if (t) atomicAdd(cnt_dst, p.count > 1 ? t * (unsigned long long)p.count : t);
    }
  }
}

template <int BM, int BN, int WM, int WN, int KB, class Op, int SWZ, int PREF = 1>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
k_nt_step(NTParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  if (step_is_done(p)) return;
  int tm, tn;
  tile_coords(blockIdx.x, gridDim.x, p.tiles_m, p.tiles_n, tm, tn);
  nt_tile<BM, BN, WM, WN, KB, Op, SWZ, PREF>(p, tm * BM, tn * BN, p.count ? p.ones + (p.step % kRing) : nullptr,
                                             smem, (int)threadIdx.x);
}

// ----------------------------------------------------------------- small relations
// Whole-K tiles for small n: a 32 x 32 output tile per workgroup whose 32 rows
// of X and 32 rows of Y are fetched completely into LDS at once
// (global_load_lds_dwordx4, all issued before the first wait), so the product
// waits on memory once instead of once per K slice.  Sixteen waves: four
// groups of four, each wave of a group owning one 16 x 16 block of the tile,
// group k taking every fourth K step from step k (four waves per SIMD hide
// the LDS latency of the K loop); groups 1..3 leave their partial sums in
// LDS and group 0 adds them (integer counts, exact also in fp32).  LDS: row
// r (X rows 0..31, then Y rows) at r * ldb, its 16-byte chunk c stored at
// c ^ (r & mask) (mask 15, or 7 when a row has fewer than 16 chunks), so the
// 16 lanes that read one chunk of 16 rows hit distinct banks; then the
// partial sums, then the epilogue tile (32 x 48 bytes).
constexpr int kSmallMaxLdb = 2048;  // largest row of operand bytes (LDS: 64 rows + the rest)
constexpr int kSmallEst = 48;
constexpr int kSmallKS = 4;                    // K groups
constexpr int kSmallThreads = 256 * kSmallKS;  // four waves per group
constexpr int kSmallPart = (kSmallKS - 1) * 4 * 64 * 16;  // groups 1..3: 4 blocks x 64 lanes x 16 B

size_t small_lds_bytes(int64_t ldb) { return (size_t)64 * ldb + kSmallPart + 32 * kSmallEst; }

// The product of a small tile: X rows 0..31 and Y rows 32..63 of the LDS
// image (chunk c of row r at c ^ (r & mask)), four K groups of four waves,
// groups 1..3 handing their partial sums to group 0 through LDS, which
// writes the 0/1 result into the epilogue tile et (32 rows of kSmallEst
// bytes).  Called by all kSmallThreads threads; ends before the barrier
// that publishes et.  With XBYTES (fp32 only) the 32 X rows are 0/1 bytes
// instead, xrow bytes per row from the start of the LDS image with the
// 16-byte chunk c of row r at c ^ (r & 15), and each lane turns the four
// bytes behind its operand chunk into four floats.
template <class Op, bool XBYTES = false>
__device__ inline void small_tile_product(uint8_t* smem, int64_t ldb, int kc, int mask, int lane, int wave,
                                          uint8_t* et, int xrow = 0) {
  static_assert(!XBYTES || Op::kPrec == P_F32, "byte-valued X rows feed the fp32 product only");
  constexpr int KSTEP_CHUNKS = (64 / Op::FR) * Op::CPL;
  const int kg = wave >> 2, wq = wave & 3;  // K group, block of the tile
  const int wm = wq >> 1, wn = wq & 1;
  const int g = lane / Op::FR, rf = lane % Op::FR;
  const int ra = 16 * wm + rf, rb = 32 + 16 * wn + rf;
  const uint8_t* xa = smem + (int64_t)ra * ldb;
  const uint8_t* yb = smem + (int64_t)rb * ldb;
  typename Op::Acc acc = Op::zero();
  const int ksteps = kc / KSTEP_CHUNKS;
  for (int ks = kg; ks < ksteps; ks += kSmallKS) {
    u32x4 a[Op::CPL], b[Op::CPL];
#pragma unroll
    for (int c = 0; c < Op::CPL; ++c) {
      const int ch = ks * KSTEP_CHUNKS + g * Op::CPL + c;
      if constexpr (XBYTES) {
        // fp32 chunk ch = 4 ks + g holds k = 16 ks + 4 g .. + 3: dword g of
        // byte chunk ks of the row
        const unsigned w = *(const unsigned*)(smem + ra * xrow + 16 * (ks ^ (ra & 15)) + 4 * g);
        const v4f f = {(float)(w & 0xffu), (float)((w >> 8) & 0xffu), (float)((w >> 16) & 0xffu), (float)(w >> 24)};
        a[c] = __builtin_bit_cast(u32x4, f);
      } else {
        a[c] = *(const u32x4*)(xa + 16 * (ch ^ (ra & mask)));
      }
      b[c] = *(const u32x4*)(yb + 16 * (ch ^ (rb & mask)));
    }
    acc = Op::mma(a, b, acc);
  }
  typename Op::Acc* part = (typename Op::Acc*)(smem + 64 * ldb);
  if (kg > 0) part[((kg - 1) * 4 + wq) * 64 + lane] = acc;
  __syncthreads();
  // group 0: the sums, as a 0/1 block into the epilogue tile
  if (kg == 0) {
#pragma unroll
    for (int k = 0; k < kSmallKS - 1; ++k) acc += part[(k * 4 + wq) * 64 + lane];
#pragma unroll
    for (int v = 0; v < Op::NI; ++v) {
      int r, c;
      Op::coord(lane, v, r, c);
      et[(16 * wm + r) * kSmallEst + 16 * wn + c] = Op::nz(acc, v) ? 1 : 0;
    }
  }
}

template <class Op>
__global__ void __launch_bounds__(kSmallThreads) k_nt_small(NTParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  if (step_is_done(p)) return;
  constexpr int NIB = elem_nibbles(Op::kPrec);
  static_assert(Op::FR == 16 && Op::NI == 4 && sizeof(typename Op::Acc) == 16, "16 x 16 blocks, 16-byte sums");
  int tm, tn;
  tile_coords(blockIdx.x, gridDim.x, p.tiles_m, p.tiles_n, tm, tn);
  const int row0 = tm * 32, col0 = tn * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ldb = p.ld * NIB / 2;
  const int kc = (int)(ldb / 16);
  const int mask = (kc % 16 == 0) ? 15 : 7;
  const uint8_t* Xg = (const uint8_t*)p.X + (int64_t)row0 * ldb;
  const uint8_t* Yg = (const uint8_t*)p.Y + (int64_t)col0 * ldb;
  // 64 * kc chunks, 64 per DMA instruction: instruction i fills LDS chunks
  // [64 i, 64 i + 64), lane L the chunk at position q = 64 i + L
  for (int i = wave; i < kc; i += kSmallThreads / 64) {
    const int q = 64 * i + lane;
    const int r = q / kc, pos = q % kc;
    const int c = pos ^ (r & mask);
    const uint8_t* src = (r < 32 ? Xg + (int64_t)r * ldb : Yg + (int64_t)(r - 32) * ldb) + 16 * c;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)(smem + 1024 * i), 16, 0, 0);
  }
  __syncthreads();  // waits for every load of this workgroup (vmcnt(0)) and joins the waves

  uint8_t* et = smem + 64 * ldb + kSmallPart;
  small_tile_product<Op>(smem, ldb, kc, mask, lane, wave, et);
  __syncthreads();
  int cnt = 0;
  uint8_t* outb = (uint8_t*)p.out;
  if (tid < 64) {  // 32 rows x two 16-byte segments
    const int r = tid >> 1, cs = tid & 1;
    u32x4 v = *(const u32x4*)(et + r * kSmallEst + 16 * cs);
    const int gr = row0 + r, gc = col0 + 16 * cs;
    if (p.add) v |= load_add16<Op::kPrec>(p, gr, gc);
    if (p.add_identity) v = with_diag(v, gr, gc, p.n_valid);
    cnt = popc16(v);
    store_bool16<Op::kPrec>(outb + ((int64_t)gr * p.ld + gc) * NIB / 2, v);
    if (p.outT) *(u32x4*)(et + r * kSmallEst + 16 * cs) = p.outT_ident ? with_diag(v, gr, gc, p.n_valid) : v;
  }
  if (p.outT) {
    __syncthreads();
    if (tid < 64) {  // column c, rows 16 rs .. 16 rs + 15
      const int c = tid & 31, rs = tid >> 5;
      u32x4 v;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint8_t* e = et + (16 * rs + 4 * w) * kSmallEst + c;
        v[w] = (unsigned)e[0] | ((unsigned)e[kSmallEst] << 8) | ((unsigned)e[2 * kSmallEst] << 16) |
               ((unsigned)e[3 * kSmallEst] << 24);
      }
      store_bool16<Op::kPrec>((uint8_t*)p.outT + ((int64_t)(col0 + c) * p.ld + row0 + 16 * rs) * NIB / 2, v);
    }
  }
  if (p.count && wave == 0) {
    cnt = wave_sum(cnt);
    if (lane == 0 && cnt) atomicAdd(p.ones + (p.step % kRing), (unsigned long long)cnt);
  }
}

template <class Op>
static hipError_t launch_small(const NTParams& p, hipStream_t s) {
  const int64_t ldb = p.ld * elem_nibbles(Op::kPrec) / 2;
  if (ldb > kSmallMaxLdb || ldb % 128 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_nt_small<Op>, dim3(p.tiles_m * p.tiles_n), dim3(kSmallThreads), small_lds_bytes(ldb), s, p);
  return hipGetLastError();
}

template <class Op>
static hipError_t set_lds_attr_small() {
  return hipFuncSetAttribute((const void*)k_nt_small<Op>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)small_lds_bytes(kSmallMaxLdb));
}

// ----------------------------------------------------------------- whole plain fixpoint in one launch
// The plain series of Sec. 3, run transposed (S = R^T): S^(1) = A^T,
// S^(t) = [S^(t-1) (A + I)^T], for Np <= 512 (operand rows of at most 2 KB),
// as one launch of one workgroup per 32 x 32 tile of S, all resident at once
// (cooperative launch).  The right operand A + I never changes: each
// workgroup builds its 32 rows of it once, from the caller's bytes, and keeps
// them in LDS; each step it fetches its 32 rows of S^(t-1) (whole K, as in
// k_nt_small) and writes its tile of S^(t).
//
// Row blocks are independent.  Block i of S^(t) (its rows 32 i .. 32 i + 31)
// is block i of S^(t-1) times (A + I)^T, so it depends on no other block,
// and once it repeats (S^(k) = S^(k-1) on those rows) it stays fixed.  The
// tiles_n workgroups of tile row i therefore run their own series: between
// steps they wait only for each other, through one word per step,
// rowstep[i][t] = arrivals + 256 x (tiles whose count changed at step t);
// the series of block i has repeated at step k_i when every tile of it is
// unchanged there (counts only grow, so "changed" = "count changed"), and
// all its workgroups stop there together.  The iterates of the whole matrix
// first repeat at K = max_i k_i; its model sizes, ones[t] = sum_i
// ones_i[min(t, k_i)], are summed by the last workgroup to finish.  A tile
// of S^(t) overwrites the same tile of S^(t-2), whose only readers (the
// workgroups of its row, in step t-1) have arrived at step t-1 before the
// writer starts step t.
//
// Coherence across XCDs without cache flushes: the tiles and counters are
// written with device-scope stores and atomics (write-through, "sc1") and
// the next step's rows fetched with device-scope loads (sc1, past any stale
// L1 or L2 copy); a workgroup waits for its tile's stores to complete
// (s_waitcnt vmcnt(0)) before it counts its arrival.
//
// Each wait polls with a time limit (s_memrealtime ticks, 100 MHz); past it
// the workgroup raises the abort word, reports it in status_out[1] and
// leaves, and every other wait sees the abort word and leaves.  On stopping,
// each workgroup writes its tile of the last iterate into the caller's R,
// transposed back and cropped to n x n.  The last workgroup to finish writes
// ring_out[0 .. K] and status_out = {K, 0}, then zeroes the counters for the
// next launch.

__device__ inline unsigned ld_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long ld_agent64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until this wave's stores and atomics have completed.
__device__ inline void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Polls *p until (*p & mask) >= target; returns the word, or ~0u on a time
// limit (then the abort word is raised and status_out[1] set) or an abort
// seen in the abort word.
__device__ inline unsigned wait_word(const unsigned* p, unsigned mask, unsigned target, unsigned* abort_word,
                                     unsigned* status_out, long long limit) {
  const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
  for (;;) {
    const unsigned w = ld_agent(p);
    if ((w & mask) >= target) return w;
    if (ld_agent(abort_word) != 0u) return ~0u;
    if ((long long)__builtin_amdgcn_s_memrealtime() - t0 > limit) {
      st_agent(abort_word, 1u);
      st_agent(status_out + 1, 1u);
      return ~0u;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Device-scope (write-through, sc1) stores of 16 and 8 bytes at byte offset
// off of a buffer (buffer instructions: the compiler knows them as stores
// and keeps the wait states their data registers need).
constexpr int kCpolSc1 = 16;  // cache-policy bits of a device-scope access
__device__ inline __amdgpu_buffer_rsrc_t buffer_of(void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
__device__ inline void st_agent_x4(__amdgpu_buffer_rsrc_t r, int off, u32x4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kCpolSc1);
}
__device__ inline void st_agent_x2(__amdgpu_buffer_rsrc_t r, int off, unsigned lo, unsigned hi) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  u32x2 v = {lo, hi};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, kCpolSc1);
}

// 16 boolean bytes as 16 operand elements (the bytes store_bool16 writes),
// stored with device-scope stores at byte offset off of buffer r.
template <int PREC>
__device__ inline void store_bool16_agent(__amdgpu_buffer_rsrc_t r, int off, u32x4 b) {
  if constexpr (PREC == P_I8) {
    st_agent_x4(r, off, b);
  } else if constexpr (PREC == P_FP8) {
    st_agent_x4(r, off, b * 0x38u);
  } else if constexpr (PREC == P_FP4) {
    unsigned w2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const unsigned x = b[2 * h], y = b[2 * h + 1];
      const unsigned lo = ((x & 1u) << 1) | (((x >> 8) & 1u) << 5) | (((x >> 16) & 1u) << 9) | (((x >> 24) & 1u) << 13);
      const unsigned hi = ((y & 1u) << 1) | (((y >> 8) & 1u) << 5) | (((y >> 16) & 1u) << 9) | (((y >> 24) & 1u) << 13);
      w2[h] = lo | (hi << 16);
    }
    st_agent_x2(r, off, w2[0], w2[1]);
  } else if constexpr (PREC == P_BF16) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u32x4 v;
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const unsigned x = b[2 * h + w];
        v[2 * w] = ((x & 1u) ? 0x3F80u : 0u) | (((x >> 8) & 1u) ? 0x3F800000u : 0u);
        v[2 * w + 1] = (((x >> 16) & 1u) ? 0x3F80u : 0u) | (((x >> 24) & 1u) ? 0x3F800000u : 0u);
      }
      st_agent_x4(r, off + 16 * h, v);
    }
  } else {  // F32
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const unsigned x = b[w];
      u32x4 v;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = ((x >> (8 * q)) & 1u) ? 0x3F800000u : 0u;
      st_agent_x4(r, off + 16 * w, v);
    }
  }
}

// 16-byte LDS chunk of operand elements from the low bits of `bits`
// (element e of the chunk set iff bit e is set; 32 / nibbles elements).
template <int PREC>
__device__ inline u32x4 chunk_of_bits(unsigned bits) {
  u32x4 v = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    unsigned x = 0u;
    if constexpr (PREC == P_F32) {
      x = ((bits >> w) & 1u) ? 0x3F800000u : 0u;
    } else if constexpr (PREC == P_BF16) {
      x = (((bits >> (2 * w)) & 1u) ? 0x3F80u : 0u) | (((bits >> (2 * w + 1)) & 1u) ? 0x3F800000u : 0u);
    } else if constexpr (PREC == P_FP4) {
#pragma unroll
      for (int q = 0; q < 8; ++q) x |= ((bits >> (8 * w + q)) & 1u) << (4 * q + 1);
    } else {
      const unsigned one = PREC == P_FP8 ? 0x38u : 1u;
#pragma unroll
      for (int q = 0; q < 4; ++q) x |= ((bits >> (4 * w + q)) & 1u) ? one << (8 * q) : 0u;
    }
    v[w] = x;
  }
  return v;
}

template <class Op>
__global__ void __launch_bounds__(kSmallThreads) k_fix_small(FixSmallParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  __shared__ int s_go;  // 1 compute the step, 0 stop, -1 abort
  // fp32: the iterates are kept as 0/1 bytes (Np bytes per row) and widened
  // to floats as the product reads them, so that a step publishes and
  // fetches a quarter of the bytes
  constexpr bool XB = Op::kPrec == P_F32;
  constexpr int NIB = elem_nibbles(Op::kPrec);
  constexpr int EPC = 32 / NIB;  // operand elements per 16-byte chunk
  const unsigned G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, (int)G);  // XCD-contiguous runs of tile rows
  const int ti = L / p.tiles, tj = L % p.tiles;
  const int row0 = 32 * ti, col0 = 32 * tj;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ldb = (int64_t)p.Np * NIB / 2;
  const int kc = (int)(ldb / 16);
  const int mask = (kc % 16 == 0) ? 15 : 7;
  const int stride = p.Np + 3;  // entries per row block in rowstep and ones_row
  unsigned* rowstep = p.rowstep + (int64_t)ti * stride;
  uint8_t* et = smem + 64 * ldb + kSmallPart;

  // One pass over rows col0 .. col0 + 31 of A builds both Y = those rows
  // of A + I (LDS rows 32..63, kept for the whole series) and S^(1) = A^T
  // (tile element (r, c) is A[col0 + c][row0 + r], i.e. the columns
  // row0 .. row0 + 31 of the same rows, before the identity is added).
  // Each item is the EPC bytes of A behind one operand chunk (consecutive
  // threads write consecutive chunks), read with one load where it is
  // aligned and inside the n valid columns, bytewise elsewhere.
  for (int q = tid; q < 32 * kc; q += kSmallThreads) {
    const int r = q / kc, c = q % kc;
    const int j = col0 + r, k0 = c * EPC;
    unsigned raw = 0u;  // bit e: A[j][k0 + e] != 0
    if (j < p.n) {
      const uint8_t* src = p.A + (int64_t)j * p.lda + k0;
      if (k0 + EPC <= p.n && ((uintptr_t)src & (EPC >= 16 ? 15 : EPC - 1)) == 0) {
        unsigned w[EPC / 4];
        if constexpr (EPC >= 16) {
#pragma unroll
          for (int h = 0; h < EPC / 16; ++h) {
            const u32x4 v = *(const u32x4*)(src + 16 * h);
#pragma unroll
            for (int x = 0; x < 4; ++x) w[4 * h + x] = v[x];
          }
        } else if constexpr (EPC == 8) {
          const uint2 v = *(const uint2*)src;
          w[0] = v.x;
          w[1] = v.y;
        } else {
          w[0] = *(const unsigned*)src;
        }
#pragma unroll
        for (int x = 0; x < EPC / 4; ++x)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if ((w[x] >> (8 * b)) & 0xffu) raw |= 1u << (4 * x + b);
      } else {
        for (int e = 0; e < EPC; ++e)
          if (k0 + e < p.n && src[e] != 0) raw |= 1u << e;
      }
    }
    // S^(1): the part of this item inside columns row0 .. row0 + 31
    if (k0 + EPC > row0 && k0 < row0 + 32)
      for (int e = 0; e < EPC; ++e) {
        const int k = k0 + e;
        if (k >= row0 && k < row0 + 32) et[(k - row0) * kSmallEst + r] = (raw >> e) & 1u;
      }
    if (j >= k0 && j < k0 + EPC && j < p.n) raw |= 1u << (j - k0);  // the identity of A + I
    *(u32x4*)(smem + (int64_t)(32 + r) * ldb + 16 * (c ^ ((32 + r) & mask))) = chunk_of_bits<Op::kPrec>(raw);
  }
  __syncthreads();

  int t = 1, prev_cnt = 0;
  for (;;) {
    // publish S^(t) from et: stores, count, then the arrival (wave 0)
    if (wave == 0) {
      const int r = lane >> 1, cs = lane & 1;
      const u32x4 v = *(const u32x4*)(et + r * kSmallEst + 16 * cs);
      if constexpr (XB)
        st_agent_x4(buffer_of(p.S[t & 1], (unsigned)(p.Np * p.Np)), (row0 + r) * p.Np + col0 + 16 * cs, v);
      else
        store_bool16_agent<Op::kPrec>(buffer_of(p.S[t & 1], (unsigned)(ldb * p.Np)),
                                      (int)(((int64_t)(row0 + r) * p.Np + col0 + 16 * cs) * NIB / 2), v);
      const int cnt = wave_sum(popc16(v));
      const unsigned changed = cnt != prev_cnt ? 1u : 0u;
      prev_cnt = cnt;
      wait_stores();
      if (lane == 0) atomicAdd(rowstep + t, 1u + (changed << 8));
      // the model size after the arrival, so the arrival does not wait for
      // it; the wait before the finishing count below covers it
      if (lane == 0 && cnt) atomicAdd(p.ones_row + (int64_t)ti * stride + t, (unsigned long long)cnt);
    }
    ++t;
    // decide whether step t runs: the row's arrivals at step t - 1
    if (tid == 0) {
      int go = 1;
      if (t > p.max_steps) {
        go = 0;
      } else {
        const unsigned w = wait_word(rowstep + (t - 1), 0xffu, (unsigned)p.tiles, p.finished + 1, p.status_out,
                                     p.wait_limit);
        if (w == ~0u) go = -1;
        else if ((w >> 8) == 0u) go = 0;  // no tile of the row changed: its series repeated at t - 1
      }
      s_go = go;
    }
    __syncthreads();
    const int go = s_go;
    if (go < 0) return;
    if (go == 0) break;
    // X = rows row0 .. row0 + 31 of S^(t-1) into LDS rows 0..31
    const int xrow = XB ? p.Np : (int)ldb;  // bytes per X row (global and LDS)
    const int xc = xrow / 16, xmask = XB ? 15 : mask;
    const uint8_t* Xg = (const uint8_t*)p.S[(t - 1) & 1] + (int64_t)row0 * xrow;
    for (int i = wave; i < xc / 2; i += kSmallThreads / 64) {
      const int q = 64 * i + lane;
      const int r = q / xc, pos = q % xc;
      const int c = pos ^ (r & xmask);
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(Xg + (int64_t)r * xrow + 16 * c),
                                       (__attribute__((address_space(3))) void*)(smem + 1024 * i), 16, 0, kCpolSc1);
    }
    __syncthreads();  // vmcnt(0): the panel is in LDS
    small_tile_product<Op, XB>(smem, ldb, kc, mask, lane, wave, et, xrow);
    __syncthreads();
  }
  // the last iterate computed, S^(t-1), back to R = S^T, cropped; every
  // store of the tile completes before the workgroup counts itself finished
  for (int q = tid; q < 1024; q += kSmallThreads) {
    const int r = q & 31, c = q >> 5;
    const int gi = row0 + r, gj = col0 + c;
    if (gi < p.n && gj < p.n) p.R[(int64_t)gj * p.ldr + gi] = et[r * kSmallEst + c];
  }
  wait_stores();
  __syncthreads();
  // the last workgroup to finish sums the model sizes of the whole matrix
  if (tid == 0) {
    if (tj == 0) st_agent(p.krow + ti, (unsigned)(t - 1));
    wait_stores();
    s_go = atomicAdd(p.finished, 1u) == G - 1 ? 1 : 0;
  }
  __syncthreads();
  if (!s_go) return;
  // every row block's last step into LDS (one load each, all in flight
  // together), then per step s the sum over row blocks of ones_i[min(s, k_i)]
  // (independent loads)
  __shared__ int s_k[kSmallMaxLdb / 32];
  if (tid < p.tiles) s_k[tid] = (int)ld_agent(p.krow + tid);
  __syncthreads();
  int K = 0;
  for (int i = 0; i < p.tiles; ++i) K = s_k[i] > K ? s_k[i] : K;
  // K <= Np + 2 < kSmallThreads: thread s sums step s
  if (tid <= K) {
    unsigned long long sum = 0ull;
    if (tid > 0)
      for (int i = 0; i < p.tiles; ++i)
        sum += ld_agent64(p.ones_row + (int64_t)i * stride + (tid < s_k[i] ? tid : s_k[i]));
    p.ring_out[tid] = sum;
  }
  __syncthreads();
  // every other workgroup is done with the counters: zero them
  const int64_t rows = (int64_t)p.tiles * stride;
  for (int64_t i = tid; i < rows; i += kSmallThreads) {
    st_agent(p.rowstep + i, 0u);
    __hip_atomic_store(p.ones_row + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (tid < p.tiles) st_agent(p.krow + tid, 0u);
  if (tid == 0) st_agent(p.finished, 0u);
  // the status word last, once every store above has completed: a caller may
  // take it as the end of the launch
  wait_stores();
  __syncthreads();
  if (tid == 0) {
    p.status_out[1] = 0u;
    p.status_out[0] = (unsigned)K;
  }
}

__global__ void k_fix_small_clear(FixSmallParams p) {
  const int64_t rows = (int64_t)p.tiles * (p.Np + 3);
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x) {
    p.rowstep[i] = 0u;
    p.ones_row[i] = 0ull;
    if (i < p.tiles) p.krow[i] = 0u;
    if (i < 2) p.finished[i] = 0u;
  }
}

template <class Op>
static hipError_t set_lds_attr_fix_small() {
  return hipFuncSetAttribute((const void*)k_fix_small<Op>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)small_lds_bytes(kSmallMaxLdb));
}

template <class Op>
static hipError_t launch_fix_small_op(FixSmallParams p, hipStream_t s) {
  const int64_t ldb = (int64_t)p.Np * elem_nibbles(Op::kPrec) / 2;
  if (ldb > kSmallMaxLdb || ldb % 128 != 0 || p.tiles * 32 != p.Np) return hipErrorInvalidValue;
  void* args[] = {&p};
  return hipLaunchCooperativeKernel((const void*)k_fix_small<Op>, dim3(p.tiles * p.tiles), dim3(kSmallThreads), args,
                                    (unsigned)small_lds_bytes(ldb), s);
}

// ----------------------------------------------------------------- grouped step (serving)
// One launch advances many independent fixpoints by one product each.  The
// work list is the concatenation of every request's 64 x 64 output tiles;
// desc[a].tile_start is the running tile count.  A persistent grid walks the
// list with a stride of gridDim.x, so every workgroup ends after at most
// ceil(total / gridDim.x) tiles.  Each pass over gridDim.x consecutive tiles
// gives every XCD a contiguous run of them (xcd_logical), so neighbouring
// tiles of one request, which read the same operand panels, share an L2.
// T x T tiles, four waves of (T/2) x (T/2): 64 for small requests, 128 for
// the others (four times the work per tile, twice the operand reuse).
// dyn_total: the live tile count after k_group_upload skipped the products of
// finished requests (their descriptors then hold no tiles), or null.
template <int T>
__global__ void __launch_bounds__(256)
k_group_step(const GroupDesc* __restrict__ desc, int nreq, int total_tiles, const int* __restrict__ dyn_total) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  if (dyn_total) total_tiles = min(total_tiles, *dyn_total);
  for (int item = xcd_logical(blockIdx.x, gridDim.x); item < total_tiles; item += gridDim.x) {
    int lo = 0, hi = nreq - 1;  // last request whose first tile is <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (desc[mid].tile_start <= item) lo = mid;
      else hi = mid - 1;
    }
    const GroupDesc& g = desc[lo];
    int local = item - g.tile_start;
    const int tiles_n = g.Np / T;
    int tm, tn;
    if (!g.sym) {
      tm = local / tiles_n;
      tn = local % tiles_n;
    } else {  // the tiles tm <= tn, row by row
      tm = 0;
      while (local >= tiles_n - tm) {
        local -= tiles_n - tm;
        ++tm;
      }
      tn = tm + local;
    }
    NTParams p{};
    p.X = g.X;
    p.Y = g.Y;
    p.ld = g.Np;
    p.Np = g.Np;
    p.add = g.add;
    p.add_identity = g.add_identity;
    p.outT_ident = g.outT_ident;
    p.n_valid = g.n_valid;
    p.out = g.out;
    p.outT = g.outT;
    if (g.sym && tm != tn) {  // the mirror image goes to out as well (it holds no identity)
      p.outT = g.out;
      p.outT_ident = 0;
      p.count = 2;
    }
    __syncthreads();  // the previous tile's epilogue is done with LDS
    int tid;  // re-derived per tile: nothing computed from it stays live across tiles
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    nt_tile<T, T, T / 2, T / 2, 64, OpI8, 2, 1>(p, tm * T, tn * T, g.cnt, smem, tid);
  }
}

__global__ void k_group_dma(const GroupDesc* __restrict__ desc, int nreq, int total_tiles,
                            const int* __restrict__ dyn_total);
size_t group_dma_lds();

hipError_t launch_group_step(int tile, const GroupDesc* desc, int nreq, int total_tiles, int grid, hipStream_t s,
                             const int* dyn_total) {
  if (nreq <= 0 || total_tiles <= 0) return hipSuccess;
  if (nreq > kMaxGroupRequests) return hipErrorInvalidValue;
  if (tile == 64) {
    typedef NTKernel<64, 64, 32, 32, 64, OpI8, 2, 1> K;
    hipLaunchKernelGGL(k_group_step<64>, dim3(grid), dim3(K::NT), K::LDS_BYTES, s, desc, nreq, total_tiles,
                       dyn_total);
  } else if (tile == 128) {
    typedef NTKernel<128, 128, 64, 64, 64, OpI8, 2, 1> K;
    hipLaunchKernelGGL(k_group_step<128>, dim3(grid), dim3(K::NT), K::LDS_BYTES, s, desc, nreq, total_tiles,
                       dyn_total);
  } else if (tile == 256) {
    hipLaunchKernelGGL(k_group_dma, dim3(grid), dim3(1024), group_dma_lds(), s, desc, nreq, total_tiles, dyn_total);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------- direct-to-LDS variant
// Same product and epilogue as k_nt_step, but the K slices are fetched with
// global_load_lds_dwordx4 (global memory straight into LDS, no staging
// registers) into a ring of NSTAGE slices, so NSTAGE - 1 slices are in
// flight while one is multiplied.  Slice layout: KB-byte rows, the 16-byte
// chunk c of row r stored at position c ^ rsw(r).  One DMA instruction of a
// wave writes 1 KB of consecutive rows in lane order, so lane l fetches row
// r0 + l / KC, chunk (l % KC) ^ rsw(row): each row is still read by KC
// adjacent lanes.  rsw is chosen so that the 16 lanes reading one MFMA
// operand (16 consecutive rows, one chunk) hit distinct banks for both 32-
// and 64-bank LDS (checked exhaustively on the host).
template <int KC>
__device__ __host__ constexpr int rsw(int r) {
  return KC == 4 ? (((r >> 1) ^ (r >> 3)) & 3) : ((r ^ (r >> 1)) & 7);
}

template <int BM, int BN, int WM, int WN, int KB, class Op, int NSTAGE>
struct DmaKernel {
  static constexpr int KC = KB / 16;
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NWAVES = WAVES_M * WAVES_N;
  static constexpr int NT = NWAVES * 64;
  static constexpr int FR = Op::FR;
  static constexpr int GROUPS = 64 / FR;
  static constexpr int FM = WM / FR, FN = WN / FR;
  static constexpr int CPL = Op::CPL;
  static constexpr int KSTEP_CHUNKS = GROUPS * CPL;
  static constexpr int KSTEPS = KC / KSTEP_CHUNKS;
  static constexpr int STAGE_BYTES = (BM + BN) * KB;
  static constexpr int ROWS_PER_DMA = 1024 / KB;                 // rows one 1 KB instruction covers
  static constexpr int DMA_PER_WAVE = (BM + BN) / ROWS_PER_DMA / NWAVES;
  static constexpr int EPAD = 16;
  static constexpr int EST = BN + EPAD;
  static constexpr size_t OPER_BYTES = (size_t)NSTAGE * STAGE_BYTES;
  static constexpr size_t EPI_BYTES = (size_t)BM * EST;
  static constexpr size_t LDS_BYTES = OPER_BYTES > EPI_BYTES ? OPER_BYTES : EPI_BYTES;
  static constexpr int NIB = elem_nibbles(Op::kPrec);  // 4-bit units per element
  // 16 x 16 fragments with whole groups of four column tiles per wave use the
  // register epilogue (operands swapped in the MFMA so that a lane holds four
  // consecutive columns of one output row); not fp8, whose 32-byte fragments
  // leave no registers for it at four waves per SIMD
  static constexpr bool SWAPPED = ((FR == 16 && FN % 4 == 0) || FR == 32) && BN == 256 && Op::kPrec != P_FP8;
  static_assert(KC == 4 || KC == 8, "64- or 128-byte slices");
  static_assert(KC % KSTEP_CHUNKS == 0, "slice must hold whole MFMA k-steps");
  static_assert(((BM + BN) / ROWS_PER_DMA) % NWAVES == 0, "DMA instructions must divide evenly");
  static_assert((NSTAGE - 2) * DMA_PER_WAVE < 64, "vmcnt range");
  static_assert((BM * BN / 16) % NT == 0, "epilogue segments must divide evenly");
};

// Workgroup barrier that orders this wave's LDS accesses only: global
// stores and direct-to-LDS loads in flight stay in flight (__syncthreads
// would wait for every one of them).  The memory clobber keeps the compiler
// from moving memory accesses across it.  For LDS data written by plain LDS
// stores; data that arrives by direct-to-LDS loads needs wait_vmcnt first.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// s_waitcnt with vmcnt = N and no wait on the other counters (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Register epilogue of the direct-to-LDS kernel.  With the MFMA operands
// swapped, item v of lane (g, c) = (lane / 16, lane % 16) in 16 x 16 tile
// (i, j) is C[row WM wm + 16 i + c][col WN wn + 16 j + 4 g + v], so a lane
// holds four consecutive bytes of one output row.  Four lanes (g = 0..3,
// same c) hold a row's 64 bytes over the column tiles 4q .. 4q + 3; a 4 x 4
// dword transpose across them (permlane swaps of 16-lane rows) leaves lane g with
// the 16 bytes of tile 4q + g, which are OR-ed with the addend and stored
// straight to global memory (16 rows x 64 contiguous bytes per instruction).
// 32 x 32 tiles need only one exchange of two dwords between lanes l and
// l + 32 (32 rows x 32 bytes per instruction).  For the
// transposed copy the segments also go to LDS (chunk m of row r at chunk
// m ^ h(r), h(r) = (r ^ (r >> 4)) & 15: conflict-free for the 16-byte
// writes and the dword reads below); each thread then reads a 16 x 4 byte
// block as 16 dwords, transposes it in registers with byte permutes and
// stores four 16-byte segments of out^T.  Returns this thread's ones.
__device__ inline int ep_swz(int r) { return (r ^ (r >> 4)) & 15; }

// The four 0/1 bytes of an accumulator fragment (element i of a lane ->
// byte i): counts are non-negative, so an integer count becomes its byte by
// min(count, 1), which v_min_u32 with a byte destination select writes
// straight into byte i (SDWA, the other bytes kept): four instructions per
// fragment, where the compiler makes a compare, a select and an OR of each.
template <class Op>
__device__ inline unsigned pack_nz4(const typename Op::Acc& a) {
  if constexpr (__is_same(typename Op::Acc, v4i)) {
    const unsigned one = 1u;
    unsigned r;
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:BYTE_0 dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:DWORD"
        : "=v"(r) : "v"(a[0]), "v"(one));
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:BYTE_1 dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"
        : "+v"(r) : "v"(a[1]), "v"(one));
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:BYTE_2 dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"
        : "+v"(r) : "v"(a[2]), "v"(one));
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"
        : "+v"(r) : "v"(a[3]), "v"(one));
    return r;
  } else {
    return (Op::nz(a, 0) ? 1u : 0u) | (Op::nz(a, 1) ? 0x100u : 0u) | (Op::nz(a, 2) ? 0x10000u : 0u) |
           (Op::nz(a, 3) ? 0x1000000u : 0u);
  }
}

// HAS_ADD: p.add is set.  Without an addend no global load is issued here,
// so nothing in the epilogue waits on memory (a next tile's first slice
// prefetched just before it stays in flight).
template <class K, class Op, bool HAS_ADD>
__device__ inline int dma_epilogue_swapped(const NTParams& p, const typename Op::Acc (&acc)[K::FM][K::FN],
                                           uint8_t* et, int row0, int col0, int wm, int wn, int lane, int tid) {
  static_assert((K::FR == 16 && Op::NI == 4) || (K::FR == 32 && Op::NI == 16), "16 x 16 or 32 x 32 fragments");
  constexpr int BM = K::WAVES_M * K::FM * K::FR, BN = K::WAVES_N * K::FN * K::FR;
  constexpr int CHUNKS = BN / 16;
  static_assert(CHUNKS == 16, "the LDS swizzle assumes 256-byte tile rows");
  uint8_t* outb = (uint8_t*)p.out;
  int cnt = 0;
  // Output segment e of this lane: row lr, columns lc .. lc + 15 of the tile.
  constexpr int NSEG = K::FR == 16 ? K::FM * (K::FN / 4) : K::FM * K::FN;
  auto seg_row = [&](int e) {
    return K::FR == 16 ? wm * (K::FM * 16) + 16 * (e / (K::FN / 4)) + (lane & 15)
                       : wm * (K::FM * 32) + 32 * (e / K::FN) + (lane & 31);
  };
  auto seg_col = [&](int e) {
    return K::FR == 16 ? wn * (K::FN * 16) + 16 * (4 * (e % (K::FN / 4)) + (lane >> 4))
                       : wn * (K::FN * 32) + 32 * (e % K::FN) + 16 * (lane >> 5);
  };
  // every addend segment is requested before the first is needed, so the
  // tile waits on one memory round trip instead of one per segment
  u32x4 addv[NSEG];
#pragma unroll
  for (int e = 0; e < NSEG; ++e) {
    addv[e] = u32x4{0u, 0u, 0u, 0u};
    if constexpr (HAS_ADD) addv[e] = load_add16<Op::kPrec>(p, row0 + seg_row(e), col0 + seg_col(e));
  }
  // Only tiles that the diagonal crosses take the identity (a uniform
  // branch: the per-byte test costs every other tile nothing).
  const bool diag = row0 < col0 + BN && col0 < row0 + BM;
  const bool add_id = p.add_identity && diag, outT_id = p.outT_ident && diag;
  // one 16-byte output segment at dst: addend, identity, count, store, LDS
  // copy (with the identity when the transposed copy is the next step's Y)
  auto emit = [&](u32x4 v, int e, uint8_t* dst) {
    const int lr = seg_row(e), lc = seg_col(e);
    const int gr = row0 + lr, gc = col0 + lc;
    if constexpr (HAS_ADD) v |= addv[e];
    if (add_id) v = with_diag(v, gr, gc, p.n_valid);
    cnt += popc16(v);
    store_bool16<Op::kPrec>(dst, v);
    if (p.outT) *(u32x4*)(et + lr * BN + 16 * ((lc >> 4) ^ ep_swz(lr))) = outT_id ? with_diag(v, gr, gc, p.n_valid) : v;
  };
  if constexpr (K::FR == 16) {
    // segment (i, q) lies 16 i rows and 64 q columns from segment (0, 0):
    // one 64-bit product per tile, then uniform offsets
    uint8_t* const seg00 = outb + ((int64_t)(row0 + seg_row(0)) * p.ld + col0 + seg_col(0)) * K::NIB / 2;
    const int64_t rstep = (int64_t)16 * p.ld * K::NIB / 2;
#pragma unroll
    for (int i = 0; i < K::FM; ++i) {
#pragma unroll
      for (int q = 0; q < K::FN / 4; ++q) {
        // P[t]: the four 0/1 bytes this lane holds of column tile 4 q + t
        unsigned P[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) P[t] = pack_nz4<Op>(acc[i][4 * q + t]);
        // 4 x 4 dword transpose over the lane rows g = lane / 16 (lane g
        // then holds the 16 bytes of column tile 4 q + g): swap the odd
        // 16-lane rows of P[0] / P[2] with the even rows of P[1] / P[3],
        // then rows 2-3 of P[0] / P[1] with rows 0-1 of P[2] / P[3]
        // (v_permlane16_swap / v_permlane32_swap, no LDS round trip)
        const auto s01 = __builtin_amdgcn_permlane16_swap(P[0], P[1], false, false);
        const auto s23 = __builtin_amdgcn_permlane16_swap(P[2], P[3], false, false);
        const auto s02 = __builtin_amdgcn_permlane32_swap(s01[0], s23[0], false, false);
        const auto s13 = __builtin_amdgcn_permlane32_swap(s01[1], s23[1], false, false);
        emit(u32x4{s02[0], s13[0], s02[1], s13[1]}, i * (K::FN / 4) + q, seg00 + i * rstep + q * 64 * K::NIB / 2);
      }
    }
  } else {
    // 32 x 32 fragments: item 4 q + b of lane (h, r) = (lane / 32, lane % 32)
    // is C[row 32 i + r][column 32 j + 8 q + 4 h + b]; lanes r and r + 32
    // swap two dwords so that lane h holds columns 16 h .. 16 h + 15
    const int h = lane >> 5;
#pragma unroll
    for (int i = 0; i < K::FM; ++i) {
#pragma unroll
      for (int j = 0; j < K::FN; ++j) {
        const auto& a = acc[i][j];
        unsigned D[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          D[q] = (Op::nz(a, 4 * q) ? 1u : 0u) | (Op::nz(a, 4 * q + 1) ? 0x100u : 0u) |
                 (Op::nz(a, 4 * q + 2) ? 0x10000u : 0u) | (Op::nz(a, 4 * q + 3) ? 0x1000000u : 0u);
        const unsigned r0 = (unsigned)__shfl_xor((int)(h ? D[0] : D[2]), 32, 64);
        const unsigned r1 = (unsigned)__shfl_xor((int)(h ? D[1] : D[3]), 32, 64);
        const u32x4 v = h ? u32x4{r0, D[2], r1, D[3]} : u32x4{D[0], r0, D[1], r1};
        const int e = i * K::FN + j;
        emit(v, e, outb + ((int64_t)(row0 + seg_row(e)) * p.ld + col0 + seg_col(e)) * K::NIB / 2);
      }
    }
  }
  if (p.outT) {
    lds_barrier();  // the staged tile; the next tile's prefetched slice may stay in flight
    uint8_t* outt = (uint8_t*)p.outT;
    constexpr int RB = BM / 16, CB = BN / 4;
    for (int blk = tid; blk < RB * CB; blk += K::NT) {
      const int x = blk & 3, rb = (blk >> 2) % RB, w = (blk >> 2) / RB;
      const int cb = 4 * w + x;  // dword column: tile columns 4 cb .. 4 cb + 3
      unsigned d[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int lr = 16 * rb + k;
        d[k] = *(const unsigned*)(et + lr * BN + 16 * ((cb >> 2) ^ ep_swz(lr)) + 4 * x);
      }
      // row 4 cb + qq of out^T, columns 16 rb .. 16 rb + 15 of the tile
      uint8_t* const trow = outt + ((int64_t)(col0 + 4 * cb) * p.ld + row0 + 16 * rb) * K::NIB / 2;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        // byte qq of d[k] is element (row 16 rb + k, column 4 cb + qq); the
        // selectors put it in byte k % 4 of dword k / 4 and zero the rest
        // (selector byte 0x0c gives 0x00)
        const unsigned sel_lo = (unsigned)qq | ((unsigned)(4 + qq) << 8) | 0x0c0c0000u;
        const unsigned sel_hi = 0x0c0cu | ((unsigned)qq << 16) | ((unsigned)(4 + qq) << 24);
        u32x4 t;
#pragma unroll
        for (int m = 0; m < 4; ++m)
          t[m] = __builtin_amdgcn_perm(d[4 * m + 1], d[4 * m], sel_lo) |
                 __builtin_amdgcn_perm(d[4 * m + 3], d[4 * m + 2], sel_hi);
        store_bool16<Op::kPrec>(trow + (int64_t)qq * p.ld * K::NIB / 2, t);
      }
    }
  }
  return cnt;
}

// Persistent grid of the direct-to-LDS step: the device's compute units,
// rounded down to a multiple of 8 (set by bool_kernels_init).
static int g_cus = 256;

// Operand panels of the tile a persistent workgroup takes next: X from its
// first output row, Y from its first output column, row pitch in bytes.
struct DmaPanels {
  const uint8_t* X = nullptr;
  const uint8_t* Y = nullptr;
  int64_t ldb = 0;
};

// One BM x BN output tile (tm, tn) of the direct-to-LDS product; the whole
// workgroup calls it.  smem holds the LDS ring (and the epilogue tile).
// A persistent caller may pass the panels of its next tile: once this tile's
// last slice is being multiplied, the next tile's first slice is fetched into
// ring slot 0 and the epilogue stages its transpose in slot 1, so that fetch
// overlaps the epilogue.  Returns whether it did; the caller passes that as
// `pre` for the next tile, whose slice 0 is then already in flight.
// tid is threadIdx.x (a persistent caller passes it through an opaque move
// each tile, so that nothing derived from it is kept live across tiles).
// SK: the stream-K part of a symmetric product (k_nt_dma_sk): only the K
// slices sk->kb .. sk->ke - 1 of the tile, finished by dma_epilogue_sk.
struct SkTile {
  int t;       // upper-triangle tile index
  int kb, ke;  // K slices of this part
  int my, nc;  // this workgroup's contributor index, contributors of the tile
};
template <class K, class Op>
__device__ int dma_epilogue_sk(const NTParams& p, const SkParams& q, const typename Op::Acc (&acc)[K::FM][K::FN],
                               uint8_t* et, int row0, int col0, int wm, int wn, int lane, int tid, const SkTile& sk,
                               bool diag_tile);
template <int BM, int BN, int WM, int WN, int KB, class Op, int NSTAGE, bool SK = false>
__device__ __forceinline__ bool nt_dma_tile(const NTParams& p, int tm, int tn, uint8_t* smem, int tid,
                                            bool pre = false, DmaPanels next = DmaPanels(),
                                            const SkTile* sk = nullptr, const SkParams* skq = nullptr) {
  typedef DmaKernel<BM, BN, WM, WN, KB, Op, NSTAGE> K;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / K::WAVES_N, wn = wave % K::WAVES_N;
  const int row0 = tm * BM, col0 = tn * BN;
  const int64_t ldb = p.ld * K::NIB / 2;
  const int kb = SK ? sk->kb : 0;
  const uint8_t* Xg = (const uint8_t*)p.X + (int64_t)row0 * ldb + (int64_t)kb * KB;
  const uint8_t* Yg = (const uint8_t*)p.Y + (int64_t)col0 * ldb + (int64_t)kb * KB;
  const int nk = SK ? sk->ke - kb : (int)(ldb / KB);

  // per-lane source address of DMA instruction j of this wave in panels
  // (Xb, Yb) of row pitch lb
  auto lane_src = [&](const uint8_t* Xb, const uint8_t* Yb, int64_t lb, int j) {
    const int r = (wave + j * K::NWAVES) * K::ROWS_PER_DMA + lane / K::KC;  // X rows then Y rows
    const int c = (lane % K::KC) ^ rsw<K::KC>(r);
    return ((r < BM) ? (Xb + (int64_t)r * lb) : (Yb + (int64_t)(r - BM) * lb)) + c * 16;
  };
  // Instruction j of this wave reads rows r0 + j NWAVES ROWS_PER_DMA of the
  // X panel then the Y panel at the same chunk c (rsw repeats every 32
  // rows): one lane offset and a uniform base per instruction, so the
  // addresses take one register instead of one pointer per instruction.
  static_assert((K::NWAVES * K::ROWS_PER_DMA) % 32 == 0, "the row swizzle must repeat across instructions");
  const int r0 = wave * K::ROWS_PER_DMA + lane / K::KC;
  const unsigned lane_off = (unsigned)(r0 * ldb + 16 * ((lane % K::KC) ^ rsw<K::KC>(r0)));
  auto base_of = [&](const uint8_t* Xb, const uint8_t* Yb, int64_t lb, int j) {
    const int jr = j * K::NWAVES * K::ROWS_PER_DMA;  // uniform
    return jr < BM ? Xb + (int64_t)jr * lb : Yb + (int64_t)(jr - BM) * lb;
  };
  // the next tile's slice 0 goes to slot 0 while this tile's last slice
  // (slot 1: nk even) is multiplied and its epilogue uses slot 1
  constexpr bool CAN_PREFETCH = K::SWAPPED && NSTAGE == 2 && (size_t)BM * BN <= K::STAGE_BYTES;
  const bool prefetch = CAN_PREFETCH && next.X != nullptr && nk % 2 == 0;
  auto issue = [&](int kt) {
    uint8_t* stage = smem + (kt % NSTAGE) * K::STAGE_BYTES;
#pragma unroll
    for (int j = 0; j < K::DMA_PER_WAVE; ++j) {
      uint8_t* dst = stage + (wave + j * K::NWAVES) * 1024;  // wave-uniform
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(base_of(Xg, Yg, ldb, j) + (int64_t)kt * KB + lane_off),
          (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };
  // the next tile's slice 0 into slot 0
  auto issue_next0 = [&]() {
#pragma unroll
    for (int j = 0; j < K::DMA_PER_WAVE; ++j)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)lane_src(next.X, next.Y, next.ldb, j),
                                       (__attribute__((address_space(3))) void*)(smem + (wave + j * K::NWAVES) * 1024),
                                       16, 0, 0);
  };

  typename Op::Acc acc[K::FM][K::FN];
#pragma unroll
  for (int i = 0; i < K::FM; ++i)
#pragma unroll
    for (int j = 0; j < K::FN; ++j) acc[i][j] = Op::zero();

  const int g = lane / K::FR, rf = lane % K::FR;
  typedef u32x4 FragA[K::FM][K::CPL];
  typedef u32x4 FragB[K::FN][K::CPL];
  auto load_frags = [&](const uint8_t* xs, const uint8_t* ys, int ks, FragA& af, FragB& bf) {
#pragma unroll
    for (int i = 0; i < K::FM; ++i)
#pragma unroll
      for (int c = 0; c < K::CPL; ++c) {
        const int ch = ks * K::KSTEP_CHUNKS + g * K::CPL + c;
        const int r = wm * WM + i * K::FR + rf;
        af[i][c] = *(const u32x4*)(xs + r * KB + 16 * (ch ^ rsw<K::KC>(r)));
      }
#pragma unroll
    for (int j = 0; j < K::FN; ++j)
#pragma unroll
      for (int c = 0; c < K::CPL; ++c) {
        const int ch = ks * K::KSTEP_CHUNKS + g * K::CPL + c;
        const int r = wn * WN + j * K::FR + rf;
        bf[j][c] = *(const u32x4*)(ys + r * KB + 16 * (ch ^ rsw<K::KC>(r)));
      }
  };
  // the fragments of k-step ks + 1 are requested before the products of ks
  auto compute = [&](int buf) {
    const uint8_t* xs = smem + buf * K::STAGE_BYTES;
    const uint8_t* ys = xs + BM * KB;
    FragA af[2];
    FragB bf[2];
    load_frags(xs, ys, 0, af[0], bf[0]);
#pragma unroll
    for (int ks = 0; ks < K::KSTEPS; ++ks) {
      if (ks + 1 < K::KSTEPS) load_frags(xs, ys, ks + 1, af[(ks + 1) & 1], bf[(ks + 1) & 1]);
#pragma unroll
      for (int i = 0; i < K::FM; ++i)
#pragma unroll
        for (int j = 0; j < K::FN; ++j) {
          if constexpr (K::SWAPPED)
            acc[i][j] = Op::mma(bf[ks & 1][j], af[ks & 1][i], acc[i][j]);  // tile of C^T
          else
            acc[i][j] = Op::mma(af[ks & 1][i], bf[ks & 1][j], acc[i][j]);
        }
    }
  };

  // Two slots of two MFMA k-steps: the barrier that makes slice kt + 1
  // visible is taken in the middle of slice kt's products -- after the
  // first k-step -- and the second k-step's products (their fragments read
  // before it) are issued after it, just before the waves fetch slice
  // kt + 1's fragments.  The matrix cores then have queued work while all
  // 16 waves read LDS at once, instead of idling behind every barrier
  // (barrier after half of the second k-step, after three quarters of it,
  // or in the middle of the first: 0.3 - 4% slower at N = 8192).
  constexpr bool SPLIT = NSTAGE == 2 && K::KSTEPS == 2 && Op::kPrec != P_FP4;  // fp4 would spill registers
  auto products = [&](const FragA& a, const FragB& b, int j0, int j1) {
#pragma unroll
    for (int i = 0; i < K::FM; ++i)
#pragma unroll
      for (int j = j0; j < j1; ++j) {
        if constexpr (K::SWAPPED)
          acc[i][j] = Op::mma(b[j], a[i], acc[i][j]);  // tile of C^T
        else
          acc[i][j] = Op::mma(a[i], b[j], acc[i][j]);
      }
  };
  if constexpr (SPLIT) {
    // prologue: slice 0 (already in flight when the previous tile fetched
    // it).  A prefetched slice 0 means slot 1 is free already -- the
    // caller's barrier retired the previous epilogue's LDS use -- so slice 1
    // goes out before the wait, and its fetch overlaps the drain of the
    // previous tile's stores (which the wait for slice 0 includes): 3%
    // faster at N = 8192, four tiles per workgroup
    if (!pre) {
      issue(0);
      wait_vmcnt<0>();
    } else if (1 < nk) {
      issue(1);
      wait_vmcnt<K::DMA_PER_WAVE>();
    } else {
      wait_vmcnt<0>();
    }
    __builtin_amdgcn_s_barrier();
    if (!pre && 1 < nk) issue(1);
    for (int kt = 0; kt < nk; ++kt) {
      const uint8_t* xs = smem + (kt & 1) * K::STAGE_BYTES;
      FragA fa0, fa1;
      FragB fb0, fb1;
      load_frags(xs, xs + BM * KB, 0, fa0, fb0);
      load_frags(xs, xs + BM * KB, 1, fa1, fb1);
      products(fa0, fb0, 0, K::FN);
      if (kt + 1 < nk) {
        // slice kt + 1, issued one barrier ago, is this wave's only load in
        // flight; the barrier extends its arrival to every wave and, with
        // every LDS read of this wave retired first, frees slot kt % 2
        wait_vmcnt<0>();
        lds_barrier();
        if (kt + 2 < nk) issue(kt + 2);
        else if (prefetch) issue_next0();  // kt + 2 == nk: the next tile's slice 0, slot 0 (nk even)
      }
      products(fa1, fb1, 0, K::FN);
    }
  } else {
  // prologue: NSTAGE - 1 slices in flight (slice 0 may be in flight already;
  // then, with two slots, slot 1 is free and slice 1 goes out at once, as in
  // the split loop)
#pragma unroll
  for (int s0 = 0; s0 < NSTAGE - 1; ++s0)
    if (s0 < nk && !(pre && s0 == 0)) issue(s0);
  const bool early1 = NSTAGE == 2 && pre && 1 < nk;
  if (early1) issue(1);
  for (int kt = 0; kt < nk; ++kt) {
    // this wave's DMA for slice kt has landed once at most the later
    // slices' instructions are outstanding; the barrier extends that to
    // every wave, and also retires all reads of the slot refilled below
    if (kt == 0 && early1) wait_vmcnt<K::DMA_PER_WAVE>();
    else if (kt + NSTAGE - 2 < nk) wait_vmcnt<(NSTAGE - 2) * K::DMA_PER_WAVE>();
    else wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (kt + NSTAGE - 1 < nk && !(kt == 0 && early1)) issue(kt + NSTAGE - 1);
    if (prefetch && kt == nk - 1) issue_next0();
    compute(kt % NSTAGE);
  }
  }
  if (prefetch) {
    __builtin_amdgcn_s_barrier();  // every wave is done reading slot 1; the next slice 0 stays in flight
  } else {
    wait_vmcnt<0>();
    __syncthreads();
  }

  int cnt = 0;
  if constexpr (SK) {
    cnt = dma_epilogue_sk<K, Op>(p, *skq, acc, smem, row0, col0, wm, wn, lane, tid, *sk, tm == tn);
  } else if constexpr (K::SWAPPED) {
    uint8_t* et = prefetch ? smem + K::STAGE_BYTES : smem;
    cnt = p.add ? dma_epilogue_swapped<K, Op, true>(p, acc, et, row0, col0, wm, wn, lane, tid)
                : dma_epilogue_swapped<K, Op, false>(p, acc, et, row0, col0, wm, wn, lane, tid);
  } else {
    // ---- epilogue of k_nt_step: the 0/1 tile through LDS byte by byte
    constexpr int SEG_PER_ROW = BN / 16;
    constexpr int SEGS = BM * SEG_PER_ROW / K::NT;
    u32x4 addv[SEGS];  // addend segments, requested together as in nt_tile
#pragma unroll
    for (int i = 0; i < SEGS; ++i) {
      const int q = tid + i * K::NT;
      addv[i] = u32x4{0u, 0u, 0u, 0u};
      if (p.add) addv[i] = load_add16<Op::kPrec>(p, row0 + q / SEG_PER_ROW, col0 + (q % SEG_PER_ROW) * 16);
    }
    uint8_t* et = smem;
#pragma unroll
    for (int i = 0; i < K::FM; ++i)
#pragma unroll
      for (int j = 0; j < K::FN; ++j)
#pragma unroll
        for (int v = 0; v < Op::NI; ++v) {
          int r, c;
          Op::coord(lane, v, r, c);
          et[(wm * WM + i * K::FR + r) * K::EST + wn * WN + j * K::FR + c] = Op::nz(acc[i][j], v) ? 1 : 0;
        }
    __syncthreads();

    uint8_t* outb = (uint8_t*)p.out;
#pragma unroll
    for (int i = 0; i < SEGS; ++i) {
      const int q = tid + i * K::NT;
      const int r = q / SEG_PER_ROW, cs = q % SEG_PER_ROW;
      u32x4 v = *(const u32x4*)(et + r * K::EST + cs * 16);
      const int gr = row0 + r, gc = col0 + cs * 16;
      v |= addv[i];
      if (p.add_identity) v = with_diag(v, gr, gc, p.n_valid);
      cnt += popc16(v);
      store_bool16<Op::kPrec>(outb + ((int64_t)gr * p.ld + gc) * K::NIB / 2, v);
      if (p.outT) *(u32x4*)(et + r * K::EST + cs * 16) = p.outT_ident ? with_diag(v, gr, gc, p.n_valid) : v;
    }
    if (p.outT) {
      __syncthreads();
      constexpr int SEG_PER_COL = BM / 16;
      constexpr int TSEGS = BN * SEG_PER_COL / K::NT;
      uint8_t* outt = (uint8_t*)p.outT;
#pragma unroll 2
      for (int i = 0; i < TSEGS; ++i) {
        const int q = tid + i * K::NT;
        const int c = q % BN, rs = q / BN;
        u32x4 v;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint8_t* e = et + (rs * 16 + 4 * w) * K::EST + c;
          v[w] = (unsigned)e[0] | ((unsigned)e[K::EST] << 8) | ((unsigned)e[2 * K::EST] << 16) |
                 ((unsigned)e[3 * K::EST] << 24);
        }
        store_bool16<Op::kPrec>(outt + ((int64_t)(col0 + c) * p.ld + row0 + rs * 16) * K::NIB / 2, v);
      }
    }
  }
  if (p.count) {
    __shared__ int red[K::NWAVES];
    cnt = wave_sum(cnt);
    if (lane == 0) red[wave] = cnt;
    lds_barrier();
    if (tid == 0) {
      unsigned long long t = 0;
#pragma unroll
      for (int w = 0; w < K::NWAVES; ++w) t += (unsigned long long)red[w];
      // a global (not flat) atomic: a flat one would first wait for the
      // prefetched slice, whose LDS writes it might alias; count 2: the tile
      // stands for its mirror image too
      if (t)
        __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long*)(p.ones + (p.step % kRing)),
                               t * (unsigned long long)p.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return prefetch;
}

template <int BM, int BN, int WM, int WN, int KB, class Op, int NSTAGE>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
__attribute__((amdgpu_waves_per_eu(1, ((BM / WM) * (BN / WN) + 3) / 4 > 2 ? ((BM / WM) * (BN / WN) + 3) / 4 : 2)))
k_nt_dma(NTParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  if (step_is_done(p)) return;
  // Persistent: workgroup b takes the tiles of blocks b, b + G, b + 2G, ...
  // (G = gridDim.x, a multiple of 8 when it is below the tile count, so
  // each block keeps the XCD that tile_coords assigns it) and fetches each
  // next tile's first slice during the current tile's epilogue.
  const int T = p.tiles_m * p.tiles_n;
  const int64_t ldb = p.ld * elem_nibbles(Op::kPrec) / 2;
  bool pre = false;
  for (int v = blockIdx.x; v < T; v += gridDim.x) {
    int tm, tn;
    tile_coords(v, T, p.tiles_m, p.tiles_n, tm, tn);
    DmaPanels next;
    if (v + (int)gridDim.x < T) {
      int tm2, tn2;
      tile_coords(v + gridDim.x, T, p.tiles_m, p.tiles_n, tm2, tn2);
      next.X = (const uint8_t*)p.X + (int64_t)tm2 * BM * ldb;
      next.Y = (const uint8_t*)p.Y + (int64_t)tn2 * BN * ldb;
      next.ldb = ldb;
    }
    __syncthreads();  // the previous tile's epilogue is done with LDS
    int tid;          // re-derived per tile: nothing computed from it stays live across tiles
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    pre = nt_dma_tile<BM, BN, WM, WN, KB, Op, NSTAGE>(p, tm, tn, smem, tid, pre, next);
  }
}

// Epilogue of a stream-K part (k_nt_dma_sk).  The 0/1 segments are packed as
// in dma_epilogue_swapped.  A tile with several contributors: every one
// stores its segments in its scratch slot with write-through stores, waits
// for them, and counts itself in tile_cnt[t]; the last to arrive ORs in the
// other slots (device-scope loads), clears the counter and finishes the tile:
// identity on the diagonal tile, count, stores of the tile and (off the
// diagonal) of its mirror image.  Returns the ones it adds to the model
// size (an off-diagonal tile counts for its mirror too).
template <class K, class Op>
__device__ int dma_epilogue_sk(const NTParams& p, const SkParams& q, const typename Op::Acc (&acc)[K::FM][K::FN],
                               uint8_t* et, int row0, int col0, int wm, int wn, int lane, int tid, const SkTile& sk,
                               bool diag_tile) {
  static_assert(K::FR == 16 && Op::NI == 4 && __is_same(typename Op::Acc, v4i), "int8 16 x 16 fragments");
  constexpr int BM = K::WAVES_M * K::FM * K::FR, BN = K::WAVES_N * K::FN * K::FR;
  static_assert(BM == 256 && BN == 256, "65536-byte slots");
  constexpr int NSEG = K::FM * (K::FN / 4);
  auto seg_row = [&](int e) { return wm * (K::FM * 16) + 16 * (e / (K::FN / 4)) + (lane & 15); };
  auto seg_col = [&](int e) { return wn * (K::FN * 16) + 16 * (4 * (e % (K::FN / 4)) + (lane >> 4)); };
  u32x4 vs[NSEG];
#pragma unroll
  for (int i = 0; i < K::FM; ++i) {
#pragma unroll
    for (int qq = 0; qq < K::FN / 4; ++qq) {
      unsigned P[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) P[t] = pack_nz4<Op>(acc[i][4 * qq + t]);
      const auto s01 = __builtin_amdgcn_permlane16_swap(P[0], P[1], false, false);
      const auto s23 = __builtin_amdgcn_permlane16_swap(P[2], P[3], false, false);
      const auto s02 = __builtin_amdgcn_permlane32_swap(s01[0], s23[0], false, false);
      const auto s13 = __builtin_amdgcn_permlane32_swap(s01[1], s23[1], false, false);
      vs[i * (K::FN / 4) + qq] = u32x4{s02[0], s13[0], s02[1], s13[1]};
    }
  }
  if (sk.nc > 1) {
    constexpr unsigned kSlot = BM * BN;
    __shared__ int s_last;
    const __amdgpu_buffer_rsrc_t mine = buffer_of(q.scratch + ((size_t)sk.t * q.maxc + sk.my) * kSlot, kSlot);
#pragma unroll
    for (int e = 0; e < NSEG; ++e) st_agent_x4(mine, seg_row(e) * BN + seg_col(e), vs[e]);
    wait_stores();
    __syncthreads();
    if (tid == 0) {
      const unsigned before =
          __hip_atomic_fetch_add(q.tile_cnt + sk.t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = before == (unsigned)(sk.nc - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return 0;
    for (int k = 0; k < sk.nc; ++k) {
      if (k == sk.my) continue;
      const __amdgpu_buffer_rsrc_t other = buffer_of(q.scratch + ((size_t)sk.t * q.maxc + k) * kSlot, kSlot);
#pragma unroll
      for (int e = 0; e < NSEG; ++e)
        vs[e] |= __builtin_amdgcn_raw_buffer_load_b128(other, seg_row(e) * BN + seg_col(e), 0, kCpolSc1);
    }
    if (tid == 0) st_agent(q.tile_cnt + sk.t, 0u);
  }
  uint8_t* outb = (uint8_t*)p.out;
  const bool add_id = p.add_identity && diag_tile;
  int cnt = 0;
#pragma unroll
  for (int e = 0; e < NSEG; ++e) {
    const int lr = seg_row(e), lc = seg_col(e);
    u32x4 v = vs[e];
    if (add_id) v = with_diag(v, row0 + lr, col0 + lc, p.n_valid);
    cnt += popc16(v);
    *(u32x4*)(outb + (int64_t)(row0 + lr) * p.ld + col0 + lc) = v;
    if (!diag_tile) *(u32x4*)(et + lr * BN + 16 * ((lc >> 4) ^ ep_swz(lr))) = v;
  }
  if (!diag_tile) {
    // the mirror image: element (row0 + r, col0 + c) also at (col0 + c, row0 + r)
    lds_barrier();
    constexpr int RB = BM / 16, CB = BN / 4;
    for (int blk = tid; blk < RB * CB; blk += K::NT) {
      const int x = blk & 3, rb = (blk >> 2) % RB, w = (blk >> 2) / RB;
      const int cb = 4 * w + x;
      unsigned d[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int lr = 16 * rb + k;
        d[k] = *(const unsigned*)(et + lr * BN + 16 * ((cb >> 2) ^ ep_swz(lr)) + 4 * x);
      }
      uint8_t* const trow = outb + (int64_t)(col0 + 4 * cb) * p.ld + row0 + 16 * rb;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const unsigned sel_lo = (unsigned)qq | ((unsigned)(4 + qq) << 8) | 0x0c0c0000u;
        const unsigned sel_hi = 0x0c0cu | ((unsigned)qq << 16) | ((unsigned)(4 + qq) << 24);
        u32x4 t;
#pragma unroll
        for (int m = 0; m < 4; ++m)
          t[m] = __builtin_amdgcn_perm(d[4 * m + 1], d[4 * m], sel_lo) |
                 __builtin_amdgcn_perm(d[4 * m + 3], d[4 * m + 2], sel_hi);
        *(u32x4*)(trow + (int64_t)qq * p.ld) = t;
      }
    }
  }
  return diag_tile ? cnt : 2 * cnt;
}

// Stream-K product of a symmetric result (see SkParams): workgroup g takes the
// K slices [g share, (g + 1) share) of the upper-triangle tiles laid end to
// end (each tile nk = Np / 128 slices, tiles in row-major order), in XCD-
// contiguous runs.  No workgroup waits for another.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_nt_dma_sk(NTParams p, SkParams q) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  if (step_is_done(p)) return;
  const int nk = (int)(p.ld / 128);
  const long long U = (long long)q.tiles * nk;
  const int g = xcd_logical(blockIdx.x, gridDim.x);
  const long long u1 = min(U, (long long)(g + 1) * q.share);
  for (long long u = (long long)g * q.share; u < u1;) {
    SkTile sk;
    sk.t = (int)(u / nk);
    const long long t0 = (long long)sk.t * nk;
    sk.kb = (int)(u - t0);
    sk.ke = (int)min((long long)nk, u1 - t0);
    const int first = (int)(t0 / q.share), last = (int)((t0 + nk - 1) / q.share);
    sk.my = g - first;
    sk.nc = last - first + 1;
    int tm = 0, rem = sk.t;  // the t-th tile (tm, tn), tm <= tn, row by row
    while (rem >= q.side - tm) {
      rem -= q.side - tm;
      ++tm;
    }
    __syncthreads();  // the previous part's epilogue is done with LDS
    int tid;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    nt_dma_tile<256, 256, 64, 64, 128, OpI8, 2, true>(p, tm, tm + rem, smem, tid, false, DmaPanels(), &sk, &q);
    u = t0 + sk.ke;
  }
}

bool sk_supported(int prec, int cfg_id, int64_t Np) { return prec == P_I8 && cfg_id == 0 && Np >= 256 && Np % 256 == 0; }

void sk_plan(int64_t Np, SkParams& q) {
  const int nk = (int)(Np / 128);
  q.side = (int)(Np / 256);
  q.tiles = q.side * (q.side + 1) / 2;
  const long long U = (long long)q.tiles * nk;
  // an even deal over the compute units, but no part under 8 slices (or a
  // whole tile) where there is little work
  const long long even = (U + g_cus - 1) / g_cus;
  const long long floor_share = nk < 8 ? nk : 8;
  q.share = (int)(even > floor_share ? even : floor_share);
  // a tile's nk slices meet at most (nk - 1) / share + 2 parts
  q.maxc = (nk - 1) / q.share + 2;
}

size_t sk_scratch_bytes(const SkParams& q) {
  return (size_t)q.tiles * q.maxc * 65536 + ((size_t)q.tiles * sizeof(unsigned) + 255) / 256 * 256;
}

hipError_t launch_nt_sym_sk(const NTParams& p, const SkParams& q, hipStream_t s) {
  typedef DmaKernel<256, 256, 64, 64, 128, OpI8, 2> K;
  if (p.ld % 256 || p.ld / 256 != q.side || q.share < 1 || !q.scratch || !q.tile_cnt) return hipErrorInvalidValue;
  const long long U = (long long)q.tiles * (p.ld / 128);
  const int grid = (int)((U + q.share - 1) / q.share);
  hipLaunchKernelGGL(k_nt_dma_sk, dim3(grid), dim3(K::NT), K::LDS_BYTES, s, p, q);
  return hipGetLastError();
}

// Grouped serving step with the direct-to-LDS 256 x 256 tiles (requests with
// Np a multiple of 256): one workgroup per CU walks the concatenated tile
// lists as k_group_step does, fetching each next tile's first K slice while
// it finishes the current one.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_group_dma(const GroupDesc* __restrict__ desc, int nreq, int total_tiles, const int* __restrict__ dyn_total) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  if (dyn_total) total_tiles = min(total_tiles, *dyn_total);  // see k_group_step
  // every request's first tile, in LDS: the search for a tile's request
  // takes LDS reads instead of a chain of dependent global loads
  int* first = (int*)(smem + DmaKernel<256, 256, 64, 64, 128, OpI8, 2>::LDS_BYTES);
  for (int i = threadIdx.x; i < nreq; i += blockDim.x) first[i] = desc[i].tile_start;
  __syncthreads();
  auto find = [&](int item, int lo) {  // last request whose first tile is <= item, at or after lo
    int hi = nreq - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
  };
  // tile (tm, tn) of a request's local index: row-major over all tiles, or
  // over the tiles tm <= tn of a symmetric product
  auto coords = [](int local, int nt, int sym, int& tm, int& tn) {
    if (!sym) {
      tm = local / nt;
      tn = local % nt;
      return;
    }
    tm = 0;
    while (local >= nt - tm) {
      local -= nt - tm;
      ++tm;
    }
    tn = tm + local;
  };
  bool pre = false;  // this tile's first slice is in flight already
  int item = xcd_logical(blockIdx.x, gridDim.x);
  int cur = item < total_tiles ? find(item, 0) : 0;  // the items of a workgroup only grow
  for (; item < total_tiles; item += gridDim.x) {
    const GroupDesc& g = desc[cur];
    int tm, tn;
    coords(item - g.tile_start, g.Np / 256, g.sym, tm, tn);
    DmaPanels next;
    int nxt = cur;
    if (item + (int)gridDim.x < total_tiles) {
      nxt = find(item + gridDim.x, cur);
      const GroupDesc& h = desc[nxt];
      int tm2, tn2;
      coords(item + gridDim.x - h.tile_start, h.Np / 256, h.sym, tm2, tn2);
      next.ldb = h.Np;
      next.X = (const uint8_t*)h.X + (int64_t)tm2 * 256 * h.Np;
      next.Y = (const uint8_t*)h.Y + (int64_t)tn2 * 256 * h.Np;
    }
    NTParams p{};
    p.X = g.X;
    p.Y = g.Y;
    p.ld = g.Np;
    p.Np = g.Np;
    p.add = g.add;
    p.add_identity = g.add_identity;
    p.outT_ident = g.outT_ident;
    p.n_valid = g.n_valid;
    p.out = g.out;
    p.outT = g.outT;
    p.ones = g.cnt;
    p.count = g.cnt != nullptr;
    if (g.sym && tm != tn) {  // the mirror image goes to out as well (it holds no identity)
      p.outT = g.out;
      p.outT_ident = 0;
      p.count *= 2;
    }
    p.step = 0;
    __syncthreads();  // the previous tile's epilogue is done with LDS
    int tid;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    pre = nt_dma_tile<256, 256, 64, 64, 128, OpI8, 2>(p, tm, tn, smem, tid, pre, next);
    cur = nxt;
  }
}

template <class Op, int BM, int BN, int WM, int WN, int KB, int NSTAGE>
static hipError_t launch_dma(const NTParams& p, hipStream_t s) {
  typedef DmaKernel<BM, BN, WM, WN, KB, Op, NSTAGE> K;
  // one workgroup per compute unit (a multiple of 8), or one per tile
  const int tiles = p.tiles_m * p.tiles_n;
  const int grid = tiles > g_cus ? g_cus : tiles;
  hipLaunchKernelGGL((k_nt_dma<BM, BN, WM, WN, KB, Op, NSTAGE>), dim3(grid), dim3(K::NT), K::LDS_BYTES, s, p);
  return hipGetLastError();
}

template <class Op, int BM, int BN, int WM, int WN, int KB, int NSTAGE>
static hipError_t set_lds_attr_dma() {
  typedef DmaKernel<BM, BN, WM, WN, KB, Op, NSTAGE> K;
  return hipFuncSetAttribute((const void*)k_nt_dma<BM, BN, WM, WN, KB, Op, NSTAGE>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)K::LDS_BYTES);
}

// ----------------------------------------------------------------- configurations
// cfg 0: 256x256 tile, 16 waves of 64x64, direct-to-LDS slices (large n)
// cfg 1: 128x128 tile, 4 waves of 64x64, register-staged  (medium n)
// cfg 2: 64x64 tile,   4 waves of 32x32, register-staged  (small n)
// cfg 3: int8 only, cfg 0 with the 32 x 32 x 32 MFMA instead of 16 x 16 x 64
// cfg 4: 32x32 tile, 4 waves of 16x16, whole K in LDS (rows of at most 2 KB)

template <class Op, int BM, int BN, int WM, int WN, int KB, int SWZ = (KB == 64 ? 2 : 1), int PREF = 1>
static hipError_t launch_cfg(const NTParams& p, hipStream_t s) {
  typedef NTKernel<BM, BN, WM, WN, KB, Op, SWZ, PREF> K;
  const int grid = p.tiles_m * p.tiles_n;
  hipLaunchKernelGGL((k_nt_step<BM, BN, WM, WN, KB, Op, SWZ, PREF>), dim3(grid), dim3(K::NT), K::LDS_BYTES, s, p);
  return hipGetLastError();
}

template <class Op, int BM, int BN, int WM, int WN, int KB, int SWZ = (KB == 64 ? 2 : 1), int PREF = 1>
static hipError_t set_lds_attr() {
  typedef NTKernel<BM, BN, WM, WN, KB, Op, SWZ, PREF> K;
  return hipFuncSetAttribute((const void*)k_nt_step<BM, BN, WM, WN, KB, Op, SWZ, PREF>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)K::LDS_BYTES);
}

// Large tiles: 256x256 per workgroup, 16 waves of 64x64, 128-byte K slices
// fetched straight into a 2-slice LDS ring (fp32: 64-byte slices, 4-slice
// ring), picked by sweeping tile shapes, slice depths and ring sizes at
// n = 8192.  Smaller problems use register-staged 128x128 or 64x64 tiles so
// that enough workgroups exist to fill the 256 compute units.
template <class Op>
struct BigCfg {
  static constexpr int KB = (Op::kPrec == P_F32) ? 64 : 128;
  static constexpr int NS = (Op::kPrec == P_F32) ? 4 : 2;
  typedef DmaKernel<256, 256, 64, 64, KB, Op, NS> K;
};

template <class Op>
static hipError_t launch_op(int cfg, const NTParams& p, hipStream_t s) {
  constexpr int KSMALL = (Op::CPL == 2) ? 128 : 64;
  switch (cfg) {
    case 0: return launch_dma<Op, 256, 256, 64, 64, BigCfg<Op>::KB, BigCfg<Op>::NS>(p, s);
    case 3:
      if constexpr (Op::kPrec == P_I8) return launch_dma<OpI8x32, 256, 256, 64, 64, 128, 2>(p, s);
      return hipErrorInvalidValue;
    case 4: return launch_small<Op>(p, s);
    case 1: return launch_cfg<Op, 128, 128, 64, 64, KSMALL>(p, s);
    default: return launch_cfg<Op, 64, 64, 32, 32, KSMALL>(p, s);
  }
}

template <class Op>
static hipError_t init_op() {
  constexpr int KSMALL = (Op::CPL == 2) ? 128 : 64;
  hipError_t e;
  if ((e = set_lds_attr_dma<Op, 256, 256, 64, 64, BigCfg<Op>::KB, BigCfg<Op>::NS>()) != hipSuccess) return e;
  if constexpr (Op::kPrec == P_I8)
    if ((e = set_lds_attr_dma<OpI8x32, 256, 256, 64, 64, 128, 2>()) != hipSuccess) return e;
  if ((e = set_lds_attr_small<Op>()) != hipSuccess) return e;
  if ((e = set_lds_attr_fix_small<Op>()) != hipSuccess) return e;
  if ((e = set_lds_attr<Op, 128, 128, 64, 64, KSMALL>()) != hipSuccess) return e;
  return set_lds_attr<Op, 64, 64, 32, 32, KSMALL>();
}

template <class Op>
static TileCfg cfg_of(int cfg) {
  constexpr int KSMALL = (Op::CPL == 2) ? 128 : 64;
  switch (cfg) {
    case 0: { typedef typename BigCfg<Op>::K K; return {256, 256, BigCfg<Op>::KB, K::NT, K::LDS_BYTES}; }
    case 3: { typedef DmaKernel<256, 256, 64, 64, 128, OpI8x32, 2> K; return {256, 256, 128, K::NT, K::LDS_BYTES}; }
    case 4: return {32, 32, kSmallMaxLdb, kSmallThreads, small_lds_bytes(kSmallMaxLdb)};
    case 1: { typedef NTKernel<128, 128, 64, 64, KSMALL, Op, (KSMALL == 64 ? 2 : 1)> K; return {128, 128, KSMALL, K::NT, K::LDS_BYTES}; }
    default: { typedef NTKernel<64, 64, 32, 32, KSMALL, Op, (KSMALL == 64 ? 2 : 1)> K; return {64, 64, KSMALL, K::NT, K::LDS_BYTES}; }
  }
}

// the operand ring and epilogue, then the first tile of each request (up to kMaxGroupRequests)
size_t group_dma_lds() { return DmaKernel<256, 256, 64, 64, 128, OpI8, 2>::LDS_BYTES + kMaxGroupRequests * sizeof(int); }

hipError_t bool_kernels_init() {
  hipError_t e;
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  g_cus = cus >= 8 ? cus / 8 * 8 : 8;
  if ((e = hipFuncSetAttribute((const void*)k_group_dma, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)group_dma_lds())) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_nt_dma_sk, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)DmaKernel<256, 256, 64, 64, 128, OpI8, 2>::LDS_BYTES)) != hipSuccess)
    return e;
  if ((e = init_op<OpI8>()) != hipSuccess) return e;
  if ((e = init_op<OpF32>()) != hipSuccess) return e;
  if ((e = init_op<OpBF16>()) != hipSuccess) return e;
  if ((e = init_op<OpFP8>()) != hipSuccess) return e;
  return init_op<OpFP4>();
}

TileCfg nt_config(int prec, int cfg) {
  switch (prec) {
    case P_I8: return cfg_of<OpI8>(cfg);
    case P_F32: return cfg_of<OpF32>(cfg);
    case P_BF16: return cfg_of<OpBF16>(cfg);
    case P_FP8: return cfg_of<OpFP8>(cfg);
    default: return cfg_of<OpFP4>(cfg);
  }
}

hipError_t launch_nt_step(int prec, int cfg, const NTParams& p, hipStream_t s) {
  switch (prec) {
    case P_I8: return launch_op<OpI8>(cfg, p, s);
    case P_F32: return launch_op<OpF32>(cfg, p, s);
    case P_BF16: return launch_op<OpBF16>(cfg, p, s);
    case P_FP8: return launch_op<OpFP8>(cfg, p, s);
    case P_FP4: return launch_op<OpFP4>(cfg, p, s);
    default: return hipErrorInvalidValue;
  }
}

bool fix_small_supported(int prec, int64_t np) {
  return np > 0 && np % 256 == 0 && np * elem_nibbles(prec) / 2 <= kSmallMaxLdb && np <= 512;
}

hipError_t launch_fix_small(int prec, const FixSmallParams& p, bool clear_first, hipStream_t s) {
  if (!fix_small_supported(prec, p.Np) || p.max_steps < 1 || p.max_steps > p.Np + 2) return hipErrorInvalidValue;
  if (clear_first) {
    hipLaunchKernelGGL(k_fix_small_clear, dim3(32), dim3(256), 0, s, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (prec) {
    case P_I8: return launch_fix_small_op<OpI8>(p, s);
    case P_F32: return launch_fix_small_op<OpF32>(p, s);
    case P_BF16: return launch_fix_small_op<OpBF16>(p, s);
    case P_FP8: return launch_fix_small_op<OpFP8>(p, s);
    case P_FP4: return launch_fix_small_op<OpFP4>(p, s);
    default: return hipErrorInvalidValue;
  }
}

// Padding: every dimension is a multiple of 256, which every configuration's
// tile and K slice divide.
int64_t padded_size_for(int prec, int64_t n) {
  (void)prec;
  const int64_t q = 256;
  return n <= 0 ? 0 : ((n + q - 1) / q) * q;
}

int nt_config_count(int prec) {
  (void)prec;
  return 5;
}

bool nt_config_valid(int prec, int cfg, int64_t np) {
  if (cfg == kCfgWholeFixpoint) return fix_small_supported(prec, np);
  if (cfg < 0 || cfg >= nt_config_count(prec) || np <= 0 || np % 256) return false;
  if (cfg == 3) return prec == P_I8;
  if (cfg == 4) return np * elem_nibbles(prec) / 2 <= kSmallMaxLdb;
  return true;
}

int choose_nt_config(int prec, int64_t np) {
  // whole-K 32 x 32 tiles at Np = 256 (and fp32 at 512, where each byte
  // carries the most MFMA work); beyond that they move twice the operand
  // bytes of 64 x 64 tiles and lose.  Then enough workgroups to cover the 256
  // CUs before choosing the larger tiles (measured on MI355X).
  if (np == 256 || (prec == P_F32 && np == 512)) return 4;
  if ((np / 256) * (np / 256) >= 256) return 0;
  if ((np / 128) * (np / 128) >= 128) return 1;
  return 2;
}

// ----------------------------------------------------------------- ingest / emit
// Ingest: normalise the caller's bytes (nonzero = true) into 0/1, zero-pad to
// Np x Np, and write the layouts the chosen fixpoint needs: int8 A and A^T
// and A, A^T in operand precision, the latter two optionally with the
// identity on the first n constants (ident bits 0 and 1: the right operand
// of a closure step).  Counts the ones of A.
template <int PREC>
__global__ void __launch_bounds__(256)
k_ingest(const uint8_t* __restrict__ A, int64_t lda, int n, int Np, int8_t* A8, int8_t* AT8,
         uint8_t* Aop, uint8_t* ATop, int ident, unsigned long long* ones_slot) {
  // one 128-row strip per blockIdx.y; the strip's 128 x 128 tiles are shared
  // out over gridDim.x workgroups, so the ones counter takes few atomics.
  // Each wave reads and writes whole 128-byte row segments: thread t takes
  // rows t / 8 + 32 k (k < 4), bytes 16 (t % 8) .. + 15 of the tile.  Np is
  // a multiple of 64: the last strip and tile may be 64 wide (parts beyond Np
  // are not written).
  // row pitch 132 bytes: the transposed byte reads below (lanes 16 tile rows
  // apart) spread over the banks (at most 2-way; a 144-byte pitch put 8
  // lanes on one bank); rows are written as dwords
  __shared__ __attribute__((aligned(16))) uint8_t tile[128][132];
  const int bi = blockIdx.y;
  const int tid = threadIdx.x;
  const int r0 = tid >> 3, c0 = (tid & 7) * 16;
  const int nb = (Np + 127) / 128;
  auto load = [&](int gi, int gj0) -> u32x4 {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (gi < n) {
      const uint8_t* src = A + (int64_t)gi * lda + gj0;
      if (gj0 + 16 <= n && (((uintptr_t)src) & 15) == 0) {
        // whole 16-byte segment: fold each byte's bits into its bit 0
        u32x4 x = *(const u32x4*)src;
        x |= x >> 4;
        x |= x >> 2;
        x |= x >> 1;
        v = x & 0x01010101u;
      } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const unsigned b = (gj0 + t < n && src[t] != 0) ? 1u : 0u;
          v[t >> 2] |= b << (8 * (t & 3));
        }
      }
    }
    return v;
  };
  int cnt = 0;
  for (int bj = blockIdx.x; bj < nb; bj += gridDim.x) {
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = load(bi * 128 + r0 + 32 * k, bj * 128 + c0);
    const bool col_in = bj * 128 + c0 < Np;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = r0 + 32 * k;
      if (col_in && bi * 128 + r < Np) {
        const int64_t off = (int64_t)(bi * 128 + r) * Np + bj * 128 + c0;
        if (A8) *(u32x4*)(A8 + off) = v[k];
        if (Aop)
          store_bool16<PREC>(Aop + elem_offset(PREC, off),
                             (ident & 1) ? with_diag(v[k], bi * 128 + r, bj * 128 + c0, n) : v[k]);
      }
      cnt += popc16(v[k]);  // zero outside [0, n) anyway
      if (AT8 || ATop) {
        unsigned* t = (unsigned*)&tile[r][c0];
#pragma unroll
        for (int w = 0; w < 4; ++w) t[w] = v[k][w];
      }
    }
    if (AT8 || ATop) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int rr = r0 + 32 * k;  // row of the transposed tile = column of the tile
        u32x4 t;
#pragma unroll
        for (int w = 0; w < 4; ++w)
          t[w] = (unsigned)tile[c0 + 4 * w][rr] | ((unsigned)tile[c0 + 4 * w + 1][rr] << 8) |
                 ((unsigned)tile[c0 + 4 * w + 2][rr] << 16) | ((unsigned)tile[c0 + 4 * w + 3][rr] << 24);
        if (bj * 128 + rr >= Np || bi * 128 + c0 >= Np) continue;
        const int64_t toff = (int64_t)(bj * 128 + rr) * Np + bi * 128 + c0;
        if (AT8) *(u32x4*)(AT8 + toff) = t;
        if (ATop)
          store_bool16<PREC>(ATop + elem_offset(PREC, toff),
                             (ident & 2) ? with_diag(t, bj * 128 + rr, bi * 128 + c0, n) : t);
      }
      __syncthreads();  // the tile is refilled by the next iteration
    }
  }
  if (ones_slot) {
    __shared__ int red[4];
    cnt = wave_sum(cnt);
    if ((tid & 63) == 0) red[tid >> 6] = cnt;
    __syncthreads();
    if (tid == 0) {
      const unsigned long long s = (unsigned long long)(red[0] + red[1] + red[2] + red[3]);
      if (s) atomicAdd(ones_slot, s);
    }
  }
}

hipError_t launch_ingest(int prec, const uint8_t* A, int64_t lda, int n, int Np, int8_t* A8,
                         int8_t* AT8, void* Aop, void* ATop, int ident, unsigned long long* ones_slot,
                         hipStream_t s) {
  if (Np <= 0 || Np % 64) return hipErrorInvalidValue;
  const int strips = (Np + 127) / 128;
  dim3 grid(strips < 16 ? strips : 16, strips);
  uint8_t* a = (uint8_t*)Aop;
  uint8_t* at = (uint8_t*)ATop;
  switch (prec) {
    case P_I8: hipLaunchKernelGGL(k_ingest<P_I8>, grid, dim3(256), 0, s, A, lda, n, Np, A8, AT8, a, at, ident, ones_slot); break;
    case P_F32: hipLaunchKernelGGL(k_ingest<P_F32>, grid, dim3(256), 0, s, A, lda, n, Np, A8, AT8, a, at, ident, ones_slot); break;
    case P_BF16: hipLaunchKernelGGL(k_ingest<P_BF16>, grid, dim3(256), 0, s, A, lda, n, Np, A8, AT8, a, at, ident, ones_slot); break;
    case P_FP8: hipLaunchKernelGGL(k_ingest<P_FP8>, grid, dim3(256), 0, s, A, lda, n, Np, A8, AT8, a, at, ident, ones_slot); break;
    default: hipLaunchKernelGGL(k_ingest<P_FP4>, grid, dim3(256), 0, s, A, lda, n, Np, A8, AT8, a, at, ident, ones_slot); break;
  }
  return hipGetLastError();
}

// S = identity on the first n constants, zero elsewhere (diag(x, x) facts).
template <int PREC>
__global__ void __launch_bounds__(256) k_identity(uint8_t* S, int Np, int n) {
  const int row = blockIdx.y;
  const int c = (blockIdx.x * 256 + threadIdx.x) * 16;
  if (c >= Np) return;
  u32x4 v = {0u, 0u, 0u, 0u};
  if (row < n && row >= c && row < c + 16) {
    const int b = row - c;
    v[b >> 2] = 1u << (8 * (b & 3));
  }
  store_bool16<PREC>(S + elem_offset(PREC, (int64_t)row * Np + c), v);
}

hipError_t launch_identity(int prec, void* S, int Np, int n, hipStream_t s) {
  dim3 grid((Np / 16 + 255) / 256, Np);
  uint8_t* p = (uint8_t*)S;
  switch (prec) {
    case P_I8: hipLaunchKernelGGL(k_identity<P_I8>, grid, dim3(256), 0, s, p, Np, n); break;
    case P_F32: hipLaunchKernelGGL(k_identity<P_F32>, grid, dim3(256), 0, s, p, Np, n); break;
    case P_BF16: hipLaunchKernelGGL(k_identity<P_BF16>, grid, dim3(256), 0, s, p, Np, n); break;
    case P_FP8: hipLaunchKernelGGL(k_identity<P_FP8>, grid, dim3(256), 0, s, p, Np, n); break;
    default: hipLaunchKernelGGL(k_identity<P_FP4>, grid, dim3(256), 0, s, p, Np, n); break;
  }
  return hipGetLastError();
}

// Emit: crop the padded iterate to n x n and write 0/1 bytes into the
// caller's matrix, transposing when the fixpoint ran on R^T.
template <int PREC>
__global__ void __launch_bounds__(256)
k_emit(const uint8_t* __restrict__ S, int Np, int transpose, int n, uint8_t* R, int64_t ldr) {
  __shared__ uint8_t tile[64][64 + 4];
  const int bi = blockIdx.y, bj = blockIdx.x;  // output tile (rows bi, cols bj)
  const int tid = threadIdx.x;
  if (!transpose) {
    // thread -> (row, 16-element segment) of the 64 x 64 output tile
    const int r = tid >> 2, c0 = (tid & 3) * 16;
    const int gi = bi * 64 + r, gj0 = bj * 64 + c0;
    if (gi < n) {
      uint8_t* dst = R + (int64_t)gi * ldr + gj0;
      if (gj0 + 16 <= n && (((uintptr_t)dst) & 15) == 0) {
        *(u32x4*)dst = bool16_of<PREC>(S + ((int64_t)gi * Np + gj0) * elem_nibbles(PREC) / 2);
      } else {
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (gj0 + t < n) dst[t] = (uint8_t)elem_nz<PREC>(S, (int64_t)gi * Np + gj0 + t);
      }
    }
  } else {
    // read the source tile (rows bj, cols bi) coalesced, write transposed
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = tid + t * 256;
      const int r = e >> 6, c = e & 63;
      tile[r][c] = (uint8_t)elem_nz<PREC>(S, (int64_t)(bj * 64 + r) * Np + bi * 64 + c);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = tid + t * 256;
      const int r = e >> 6, c = e & 63;
      const int gi = bi * 64 + r, gj = bj * 64 + c;
      if (gi < n && gj < n) R[(int64_t)gi * ldr + gj] = tile[c][r];
    }
  }
}

hipError_t launch_emit(int prec, const void* S, int Np, int transpose, int n, uint8_t* R,
                       int64_t ldr, hipStream_t s) {
  const int nt = (n + 63) / 64;
  dim3 grid(nt, nt);
  const uint8_t* p = (const uint8_t*)S;
  switch (prec) {
    case P_I8: hipLaunchKernelGGL(k_emit<P_I8>, grid, dim3(256), 0, s, p, Np, transpose, n, R, ldr); break;
    case P_F32: hipLaunchKernelGGL(k_emit<P_F32>, grid, dim3(256), 0, s, p, Np, transpose, n, R, ldr); break;
    case P_BF16: hipLaunchKernelGGL(k_emit<P_BF16>, grid, dim3(256), 0, s, p, Np, transpose, n, R, ldr); break;
    case P_FP8: hipLaunchKernelGGL(k_emit<P_FP8>, grid, dim3(256), 0, s, p, Np, transpose, n, R, ldr); break;
    default: hipLaunchKernelGGL(k_emit<P_FP4>, grid, dim3(256), 0, s, p, Np, transpose, n, R, ldr); break;
  }
  return hipGetLastError();
}

// Zero the ring slots of steps [s0, s0 + count) before they accumulate, and
// optionally reset the convergence state.  A kernel, not a memset, so the
// sequence stays valid under stream capture.
__global__ void k_ring_clear(unsigned long long* ones, int* conv, int s0, int count, int reset_conv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) ones[(s0 + i) % kRing] = 0ull;
  if (i == 0 && reset_conv) *conv = kNotConverged;
}

hipError_t launch_ring_clear(unsigned long long* ones, int* conv, int s0, int count, int reset_conv,
                             hipStream_t s) {
  const int threads = 256;
  const int blocks = (count + threads - 1) / threads > 0 ? (count + threads - 1) / threads : 1;
  hipLaunchKernelGGL(k_ring_clear, dim3(blocks), dim3(threads), 0, s, ones, conv, s0, count, reset_conv);
  return hipGetLastError();
}

__global__ void k_ring_set(unsigned long long* ones, int slot, unsigned long long value) {
  if (threadIdx.x == 0) ones[slot % kRing] = value;
}

hipError_t launch_ring_set(unsigned long long* ones, int slot, unsigned long long value, hipStream_t s) {
  hipLaunchKernelGGL(k_ring_set, dim3(1), dim3(64), 0, s, ones, slot, value);
  return hipGetLastError();
}

// Largest row sum of the 0/1 relation (||A||_inf, Sec. 2): one wave per row
// on a grid of at most 1024 workgroups, 16 bytes per lane where the row is
// 16-byte aligned, one atomic per workgroup (a workgroup per row with byte
// loads and an atomic each took 116 us at N = 8192).
constexpr int kRowMaxGrid = 1024;

__global__ void __launch_bounds__(256) k_row_max(const uint8_t* A, int64_t lda, int n, int* out_max) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int best = 0;
  for (int row = blockIdx.x * 4 + wave; row < n; row += gridDim.x * 4) {
    const uint8_t* r = A + (int64_t)row * lda;
    int s = 0, j0 = 0;
    if (((uintptr_t)r & 15) == 0) {
      const int nv = n / 16;
      for (int v = lane; v < nv; v += 64) {
        u32x4 x = *(const u32x4*)(r + 16 * v);
        x |= x >> 4;  // each byte's bits folded into its bit 0
        x |= x >> 2;
        x |= x >> 1;
        s += popc16(x & 0x01010101u);
      }
      j0 = 16 * nv;
    }
    for (int j = j0 + lane; j < n; j += 64) s += r[j] != 0;
    s = wave_sum(s);
    best = s > best ? s : best;
  }
  __shared__ int red[4];
  if (lane == 0) red[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int m = max(max(red[0], red[1]), max(red[2], red[3]));
    if (m) atomicMax(out_max, m);
  }
}

hipError_t launch_row_max(const uint8_t* A, int64_t lda, int n, int* out_max, hipStream_t s) {
  const int grid = (n + 3) / 4 < kRowMaxGrid ? (n + 3) / 4 : kRowMaxGrid;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL(k_row_max, dim3(grid), dim3(256), 0, s, A, lda, n, out_max);
  return hipGetLastError();
}

}  // namespace dl
