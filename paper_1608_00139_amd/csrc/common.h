// common.h -- types and helpers shared by the library's HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Precision codes, identical to dl_prec in include/dl.h.
enum Prec { P_I8 = 0, P_F32 = 1, P_BF16 = 2, P_FP8 = 3, P_FP4 = 4 };

// Slots of the per-step model-size ring kept on the device.  Step s of a
// fixpoint accumulates the number of true entries of its iterate into
// ones[s % kRing]; kRing exceeds the largest chunk of steps launched between
// two host read-backs.
constexpr int kRing = 4096;
constexpr int kNotConverged = 0x7fffffff;

// 4-bit units (nibbles) per operand element: fp4 packs two elements per
// byte, element 2t in the low nibble of byte t.
__host__ __device__ constexpr int elem_nibbles(int prec) {
  return prec == P_F32 ? 8 : (prec == P_BF16 ? 4 : (prec == P_FP4 ? 1 : 2));
}
// Byte offset of element index e, and bytes of an Np x Np operand.
__host__ __device__ constexpr int64_t elem_offset(int prec, int64_t e) { return e * elem_nibbles(prec) / 2; }
__host__ __device__ constexpr int64_t mat_bytes(int prec, int64_t np) { return np * np * elem_nibbles(prec) / 2; }

// Parameters of one boolean product step  out = [add + X * Y^T != 0].
// Closure steps need no addend: with the identity stored in Y (Y = R^T + I
// for squaring, A + I for the plain series), X Y^T = R R + R already holds
// the previous iterate; outT_ident writes the next Y that way.
struct NTParams {
  const void* X;        // [Np x Np] operand, row-major, K contiguous
  const void* Y;        // [Np x Np] operand; row j of Y is column j of the right factor
  int64_t ld;           // leading dimension of X, Y, out, outT in elements (= Np)
  int Np;               // padded size: M = N = K = Np
  const int8_t* add;    // optional addend [Np x Np], row-major: int8 0/1 (pitch Np) or, with
                        // add_op, in operand precision (pitch ld; nonzero = true)
  int add_op;           // the addend is in operand precision
  int add_identity;     // if set, OR in (i, i) for i < n_valid
  int n_valid;          // number of real constants
  void* out;            // [Np x Np] next iterate in operand precision
  void* outT;           // optional transposed copy of out
  int outT_ident;       // outT gets (i, i) for i < n_valid as well: out^T + I
  unsigned long long* ones;  // model-size ring (read for the repeat test)
  int count;            // 1: add this iterate's number of ones to ones[step % kRing]
  int* conv;            // convergence step (null: no early exit)
  int step;             // index s of the iterate this launch produces
  int check;            // 1: detect a repeat from ones[s-1] == ones[s-2]
  int tiles_m, tiles_n; // grid in tiles
};

// One request's product in a grouped (serving) launch: T x T output tiles
// of an Np x Np int8 product, Np a multiple of T.
struct GroupDesc {
  const void* X;
  const void* Y;
  const int8_t* add;
  void* out;
  void* outT;
  unsigned long long* cnt;  // ones of this product's output (null: do not count)
  int Np;
  int n_valid;
  int add_identity;
  int outT_ident;  // outT = out^T + I (see NTParams)
  int tile_start;  // first work-list index of this request
  int sym;         // the result is symmetric (same generation's S'): only the
                   // tiles tm <= tn are listed, each off-diagonal one also
                   // written mirrored into out and counted twice
  // Skip test of a product issued before the previous round's model sizes
  // were read back: the request finished in that round exactly when its
  // cumulative counter *chk equals chk_val, and then this product gets no
  // tiles (see k_group_upload).  chk null: never skipped.
  const unsigned long long* chk;
  unsigned long long chk_val;
};

// The tile lists of one serving round, in descriptor order: segment k holds
// descriptors [begin[k], begin[k + 1]) of tile size tile[k] (begin[3] = all).
struct GroupLists {
  int begin[4];
  int tile[3];
};

// One request of a grouped admission (serving): clear its buffers, write the
// identity where same generation needs S^(1) = I, zero its admission counter,
// then scatter its edge list.  clear_start / edge_start are running totals
// (16-byte units, edges) over the requests before it.
struct AdmitDesc {
  int8_t* base;            // start of the region to clear
  long long clear_units;   // 16-byte units to clear from base
  long long clear_start;
  long long ident_off;     // byte offset from base of an Np x Np identity block, -1 if none
  int8_t* M;               // scatter targets (see k_scatter_edges); M2 / MT may be null
  int8_t* M2;
  int8_t* MT;
  unsigned long long* ones;  // distinct edges counter (may be null), zeroed by the clear
  const int32_t* edges;
  long long m;
  long long edge_start;
  int n;
  int Np;
};
hipError_t launch_admit(const AdmitDesc* d, int nreq, long long total_units, long long total_edges, hipStream_t s);

// The whole plain closure fixpoint in one cooperative launch (k_fix_small in
// bool_kernels.hip): one workgroup per 32 x 32 tile of S = R^T, for
// operand rows of at most 2 KB and Np <= 512.
struct FixSmallParams {
  const uint8_t* A;
  int64_t lda;
  uint8_t* R;
  int64_t ldr;
  void* S[2];                    // iterates, Np x Np (S^(t) in S[t & 1]): fp32 as 0/1 bytes, others in operand precision
  // counters: zero when the launch starts, and left zero by a launch that
  // ends normally (the last workgroup clears them); see fix_small_words
  unsigned long long* ones_row;  // [tiles][Np + 3] model size of each row block per step
  unsigned* rowstep;             // [tiles][Np + 3] arrivals + 256 x changes per row block and step
  unsigned* krow;                // [tiles] last step of each row block
  unsigned* finished;            // [0] workgroups done, [1] abort (a wait ran past its limit)
  // outputs (device or mapped host memory), written by the last workgroup
  unsigned long long* ring_out;  // ring_out[t] = size of S^(t), t = 0 .. K
  unsigned* status_out;          // [0] K, the last step of any row block; [1] 1 after an abort
  int n, Np, tiles;              // tiles = Np / 32 per side
  int max_steps;                 // at most Np + 2
  long long wait_limit;          // ticks
};
bool fix_small_supported(int prec, int64_t np);
// Tile-configuration id that selects it for the plain series (the product
// kernels' configurations are 0 .. nt_config_count - 1; for every other use
// of the product step this id falls back to the size rule).
constexpr int kCfgWholeFixpoint = 5;
// The cooperative launch; with clear_first, a kernel that zeroes the
// counters runs before it (needed once for fresh memory and after an abort).
// Counter words (32-bit) for padded size np: fix_small_words(np), the first
// 2 tiles (np + 3) of them holding ones_row (8-byte aligned).
hipError_t launch_fix_small(int prec, const FixSmallParams& p, bool clear_first, hipStream_t s);
inline int64_t fix_small_words(int64_t np) { return 3 * (np / 32) * (np + 3) + (np / 32) + 2; }
// Points the counters of p into `words` (fix_small_words(p.Np) of them, 8-byte aligned).
inline void fix_small_place(FixSmallParams& p, unsigned* words) {
  const int64_t rows = (int64_t)p.tiles * (p.Np + 3);
  p.ones_row = (unsigned long long*)words;
  p.rowstep = words + 2 * rows;
  p.krow = p.rowstep + rows;
  p.finished = p.krow + p.tiles;
}

// Launch helpers implemented in bool_kernels.hip.
struct TileCfg {
  int bm, bn, kb, threads;
  size_t lds_bytes;
};

hipError_t launch_nt_step(int prec, int cfg_id, const NTParams& p, hipStream_t s);

// Stream-K split of a product whose result is symmetric (the same-generation
// S' = [I + T P^T]): only the tiles tm <= tn of the 256 x 256 int8 tiling are
// computed, their tiles x (Np / 128) K slices dealt to the workgroups in runs
// of `share` slices, so that every compute unit gets the same number of
// slices.  A tile split over several workgroups is finished by the last of
// them to arrive: each stores its partial 0/1 tile in scratch slot
// (t * maxc + contributor) with write-through stores and counts itself in
// tile_cnt[t]; the last ORs the others' partials (device-scope loads), adds
// the identity, counts, writes the tile and its mirror image and clears
// tile_cnt[t] for the next launch.  tile_cnt starts at zero.
struct SkParams {
  uint8_t* scratch;    // tiles * maxc slots of 65536 bytes
  unsigned* tile_cnt;  // [tiles] arrivals, zero between launches
  int side;            // tiles per side, Np / 256
  int tiles;           // side (side + 1) / 2
  int share;           // K slices per workgroup
  int maxc;            // slots per tile (contributors at most)
};
// Whether the split applies (int8 operands, the direct-to-LDS configuration,
// Np a multiple of 256), the plan for Np, and the scratch it needs (slots,
// then the counters).
bool sk_supported(int prec, int cfg_id, int64_t Np);
void sk_plan(int64_t Np, SkParams& q);
size_t sk_scratch_bytes(const SkParams& q);
hipError_t launch_nt_sym_sk(const NTParams& p, const SkParams& q, hipStream_t s);
TileCfg nt_config(int prec, int cfg_id);
int choose_nt_config(int prec, int64_t n);
int nt_config_count(int prec);  // cfg ids are 0 .. count - 1
bool nt_config_valid(int prec, int cfg, int64_t np);  // cfg usable at padded size np
hipError_t launch_hash_bool(uint8_t* M, int64_t ld, int n, int Np, unsigned seed, hipStream_t s);
hipError_t launch_publish(const unsigned long long* src, unsigned long long* dst, int n, hipStream_t s);
int64_t padded_size_for(int prec, int64_t n);

// ident: bit 0 adds the identity (first n constants) to Aop, bit 1 to ATop;
// the ones counted are those of A alone.
hipError_t launch_ingest(int prec, const uint8_t* A, int64_t lda, int n, int Np, int8_t* A8,
                         int8_t* AT8, void* Aop, void* ATop, int ident, unsigned long long* ones_slot,
                         hipStream_t s);
hipError_t launch_identity(int prec, void* S, int Np, int n, hipStream_t s);
hipError_t launch_emit(int prec, const void* S, int Np, int transpose, int n, uint8_t* R,
                       int64_t ldr, hipStream_t s);
hipError_t launch_ring_clear(unsigned long long* ones, int* conv, int s0, int count, int reset_conv,
                             hipStream_t s);
hipError_t launch_ring_set(unsigned long long* ones, int slot, unsigned long long value, hipStream_t s);
hipError_t launch_row_max(const uint8_t* A, int64_t lda, int n, int* out_max, hipStream_t s);
hipError_t launch_col_max(const uint8_t* A, int64_t lda, int n, int* out_max, hipStream_t s);
// out = (a | b | [ident] I), or its complement within the n x n constants when
// `complement` is set; int8 0/1 Np x Np operands (a, b, out, outT may be null;
// out may alias a or b).  Adds the ones of the result to *cnt if cnt is set.
hipError_t launch_bytes_op(const int8_t* a, const int8_t* b, int ident, int complement, int n, int Np, int8_t* out,
                           int8_t* outT, unsigned long long* cnt, hipStream_t s);
// Sets byte (i, j) of M (and of M2, and byte (j, i) of MT, when not null) for
// every edge (i, j) of the device list edges[2 m] with 0 <= i, j < n; adds
// the number of distinct edges to *ones.  The matrices must be zeroed.
hipError_t launch_scatter_edges(const int32_t* edges, int64_t m, int n, int Np, int8_t* M, int8_t* M2, int8_t* MT,
                                unsigned long long* ones, hipStream_t s);
hipError_t bool_kernels_init();
// Measured matrix-core throughput (operations per second) of MFMA kind 0 int8,
// 1 fp32, 2 bf16, 3 fp8, 4 fp4, 5 fp64 on the current device, or bytes per
// second of kind 6 (LDS reads, ds_read_b128) and 7 (global-to-LDS fill,
// global_load_lds_dwordx4 from 1 MB at src); kind 8 is kind 5 with AGPR
// accumulators.  `sink` must hold 256 ints (never written).
hipError_t measure_peak(int kind, int* sink, double* ops_per_s, hipStream_t s, const uint8_t* src);
// tile: 64, 128 or 256 (every request of the list has Np a multiple of it);
// at most kMaxGroupRequests requests per launch
constexpr int kMaxGroupRequests = kRing;
// dyn_total (device int, may be null): the live tile count written by
// k_group_upload; total_tiles is then the bound the grid was sized for.
hipError_t launch_group_step(int tile, const GroupDesc* desc, int nreq, int total_tiles, int grid, hipStream_t s,
                             const int* dyn_total = nullptr);
// Copy a round's descriptors from src (a device mapping of host memory) to
// dst and renumber the tiles of each segment over the products that are not
// skipped (GroupDesc::chk); totals[k] receives segment k's live tile count.
hipError_t launch_group_upload(const GroupDesc* src, GroupDesc* dst, const GroupLists& lists, int* totals,
                               hipStream_t s);

}  // namespace dl
