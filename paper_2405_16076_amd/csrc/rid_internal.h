// Internal declarations of the streaming randomized-ID library (gfx950).
//
// Everything here is private to the library; the public interface is
// include/rid.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/rid.h"
#include "omega_table.h"

namespace rid {

constexpr int kMaxEll = 512;     // sketch rows supported
constexpr int kMaxT = 256;       // basis slots supported
constexpr int kMaxBatchStreams = 4096;  // streams per batch
constexpr int kMTile = 64;       // test-matrix rows per sketch workgroup
constexpr int kOmegaRowsPerCall = 8;

// ---------------------------------------------------------------------------
// Counter-based random numbers.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit multiplies and xors, with a Weyl key schedule.
// ---------------------------------------------------------------------------
struct Words4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input xor in one v_bitop3_b32 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  return Words4{c0, c1, c2, c3};
}

// Counter word 3 of each random stream.
constexpr uint32_t kDomainOmega = 0;
constexpr uint32_t kDomainDecision = 1;
constexpr uint32_t kPruneDraw = 0xFFFFFFFFu;

// Uniform on [0,1) with 53 bits: ((x0 >> 5) 2^26 + (x1 >> 6)) 2^-53, exact.
__device__ __forceinline__ double uniform53(uint32_t x0, uint32_t x1) {
  return ((double)(x0 >> 5) * 67108864.0 + (double)(x1 >> 6)) * (1.0 / 9007199254740992.0);
}

// The decision uniform of draw (u, slot, r) of the prune/fill step.
__device__ __forceinline__ double decision_uniform(uint64_t seed, uint32_t u, uint32_t slot,
                                                   uint32_t r) {
  Words4 w = philox4x32_10(u, slot, r, kDomainDecision, (uint32_t)seed, (uint32_t)(seed >> 32));
  return uniform53(w.x, w.y);
}

// ---------------------------------------------------------------------------
// The test matrix Omega.  Entry (r, i): the Philox call with counter
// (i mod 2^32, i / 2^32, r / 8, 0) yields four words w0..w3, i.e. eight 16-bit
// halves h_{2p} = w_p & 0xFFFF, h_{2p+1} = w_p >> 16; with h = h_{r mod 8},
// Omega(r, i) = (-1)^(bit 15 of h) T[bits 14..5 of h].  T[k] is the quantile
// of |N(0,1)| at the middle of the k-th of 1024 equiprobable bins, scaled so
// that the entries have variance exactly 1 (omega_table.h): the standard
// normal quantised to 2048 equiprobable atoms.  Each form reads the table in
// its own number format, so every form holds the rounding of the same
// binary64 value, and no transcendental is evaluated on the device.
// ---------------------------------------------------------------------------

__device__ __forceinline__ Words4 omega_words(uint64_t seed, uint64_t i, uint32_t g) {
  return philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), g, kDomainOmega, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

// Half q (0..7) of the four words.
__device__ __forceinline__ uint32_t omega_half(const Words4& w, int q) {
  const uint32_t x = q < 2 ? w.x : (q < 4 ? w.y : (q < 6 ? w.z : w.w));
  return (q & 1) ? (x >> 16) : (x & 0xFFFFu);
}

__device__ __forceinline__ int omega_index(uint32_t h) { return (int)((h >> 5) & (kOmegaTabSize - 1)); }

// Copies the table of one format into LDS (every thread of the workgroup
// takes part; the caller synchronises before reading it).
template <typename T>
__device__ __forceinline__ void load_omega_table(T* lds, const T* tab) {
  constexpr int words = kOmegaTabSize * (int)sizeof(T) / 4;
  for (int i = threadIdx.x; i < words; i += blockDim.x)
    reinterpret_cast<uint32_t*>(lds)[i] = reinterpret_cast<const uint32_t*>(tab)[i];
}

// Rows 8g..8g+7 at data row i as bfloat16 bits, from an LDS copy of the table.
__device__ __forceinline__ void omega8_bf16(uint64_t seed, uint64_t i, uint32_t g, const uint16_t* tab,
                                            uint16_t z[8]) {
  const Words4 w = omega_words(seed, i, g);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t h = omega_half(w, q);
    z[q] = (uint16_t)(tab[omega_index(h)] | (h & 0x8000u));
  }
}

// The same rows from a signed copy of the bfloat16 table in LDS: entry j of
// its 2048 is T[j mod 1024] with the sign bit set for j >= 1024, so bits
// 15..5 of a half index the signed value directly.
__device__ __forceinline__ void load_omega_table_bf16_signed(uint16_t* lds) {
  for (int i = threadIdx.x; i < 2 * kOmegaTabSize; i += blockDim.x)
    lds[i] = (uint16_t)(kOmegaTabBf16[i & (kOmegaTabSize - 1)] | ((i & kOmegaTabSize) ? 0x8000u : 0u));
}

__device__ __forceinline__ void omega8_bf16_signed(uint64_t seed, uint64_t i, uint32_t g, const uint16_t* tab2,
                                                   uint16_t z[8]) {
  const Words4 w = omega_words(seed, i, g);
#pragma unroll
  for (int q = 0; q < 8; ++q) z[q] = tab2[(omega_half(w, q) >> 5) & (2 * kOmegaTabSize - 1)];
}

// A signed copy of the e4m3 table (entry j: code j mod 1024 with the sign
// bit set for j >= 1024), indexed by bits 15..5 of a half.
__device__ __forceinline__ void load_omega_table_e4m3_signed(uint8_t* lds) {
  for (int i = threadIdx.x; i < 2 * kOmegaTabSize; i += blockDim.x)
    lds[i] = (uint8_t)(kOmegaTabE4M3[i & (kOmegaTabSize - 1)] | ((i & kOmegaTabSize) ? 0x80u : 0u));
}

// Rows 8g..8g+7 at data row i as e4m3 codes of 64 Omega, from an LDS copy.
__device__ __forceinline__ void omega8_e4m3(uint64_t seed, uint64_t i, uint32_t g, const uint8_t* tab,
                                            uint32_t z[8]) {
  const Words4 w = omega_words(seed, i, g);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t h = omega_half(w, q);
    z[q] = tab[omega_index(h)] | ((h >> 8) & 0x80u);
  }
}

// Rows 8g..8g+7 at data row i in binary32 (table in device memory).
__device__ __forceinline__ void omega8_f32(uint64_t seed, uint64_t i, uint32_t g, float z[8]) {
  const Words4 w = omega_words(seed, i, g);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t h = omega_half(w, q);
    z[q] = __uint_as_float(kOmegaTabF32[omega_index(h)] | ((h & 0x8000u) << 16));
  }
}

// Rows 8g..8g+7 at data row i in binary64 (table in device memory).
__device__ __forceinline__ void omega8_f64(uint64_t seed, uint64_t i, uint32_t g, double z[8]) {
  const Words4 w = omega_words(seed, i, g);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t h = omega_half(w, q);
    const double t = kOmegaTabF64[omega_index(h)];
    z[q] = (h & 0x8000u) ? -t : t;
  }
}

// Column addresses come from a table in device memory, so the compiler cannot
// infer their address space and would emit FLAT accesses; FLAT loads also
// count against the LDS wait counter, which would make every LDS wait also
// wait for in-flight prefetches.  These casts make them global accesses.
template <typename T>
using gmem_t = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ const gmem_t<T>* gload_ptr(const T* p) {
  return (const gmem_t<T>*)p;
}

template <typename T>
__device__ __forceinline__ gmem_t<T>* gstore_ptr(T* p) {
  return (gmem_t<T>*)p;
}

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

// 16-byte global loads and stores (the address must be 16-byte aligned)
__device__ __forceinline__ float4 gload_f4(const gmem_t<float>* p) {
  const vf4 v = *reinterpret_cast<const gmem_t<vf4>*>(p);
  return make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void gstore_f4(gmem_t<float>* p, float4 x) {
  *reinterpret_cast<gmem_t<vf4>*>(p) = vf4{x.x, x.y, x.z, x.w};
}
__device__ __forceinline__ double2 gload_d2(const gmem_t<double>* p) {
  const vd2 v = *reinterpret_cast<const gmem_t<vd2>*>(p);
  return make_double2(v[0], v[1]);
}
__device__ __forceinline__ void gstore_d2(gmem_t<double>* p, double2 x) {
  *reinterpret_cast<gmem_t<vd2>*>(p) = vd2{x.x, x.y};
}

// Round-to-nearest-even binary32 -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// ---------------------------------------------------------------------------
// Device-resident state of one stream (one allocation, read and written by the
// update kernels; the host never reads it between updates).
// ---------------------------------------------------------------------------
struct DevScalars {
  int32_t nonfinite;   // 1 once a non-finite snapshot value was seen
  int32_t n_new;       // slots filled by the running update
  int32_t n_occ;       // occupied slots after the running update
  int32_t rank;        // numerical rank of Omega A_J in the running update
  int32_t pad0;
  int32_t new_slot[kMaxT];   // slots filled by the running update
  int32_t new_src[kMaxT];    // their position in the buffer
  int32_t occ_slot[kMaxT];   // occupied slots in slot order
  int32_t slot_src[kMaxT];   // buffer position of a slot filled by the running update, else -1
  int32_t old_slot[kMaxT];   // occupied slots not filled by the running update, in slot order
};

// Column j of the Gram's list: the new slots first, then the other occupied ones.
__device__ inline int gram_slot(const DevScalars* sc, int j) {
  return j < sc->n_new ? sc->new_slot[j] : sc->old_slot[j - sc->n_new];
}

// ---------------------------------------------------------------------------
// LDS-DMA staging (global_load_lds_dwordx4) shared by the streaming kernels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// Each lane copies the 16 bytes at p to LDS byte address lds_base + 16*lane
// (lds_base wave-uniform).  The copy is counted by vmcnt; the compiler does
// not see the LDS write, so the kernel waits for it explicitly.
__device__ __forceinline__ void lds_dma16(const gmem_t<float>* p, uint32_t lds_base) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(p), "s"(lds_base)
               : "memory", "m0");
}
__device__ __forceinline__ void wait_dma_keep4() { asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); }
__device__ __forceinline__ void wait_dma_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// LDS writes of this wave complete, then the workgroup barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// 16-byte slot j of a 128-byte staged column c lives at slot j ^ swz(c): the
// operand reads of 16 consecutive columns then spread over the LDS banks.
__device__ __forceinline__ int col_swz(int c) { return (c ^ (c >> 3)) & 7; }

struct SketchArgs {
  const uint64_t* colptr;  // device address of every pushed column, by global index
  int64_t c0;              // first global column of the batch
  int32_t b;               // columns in the batch
  int32_t b_max;           // column stride of a partial block
  int64_t m;               // rows per snapshot
  int64_t slab_rows;       // rows per slab (multiple of 32)
  int32_t n_slabs, n_mt, n_nt, ell_pad;
  int32_t ell;             // test-matrix rows l
  int32_t rbw;             // bf16/fp8: 32-row blocks per wave (rows per workgroup / 64);
                           // wide bf16: 32-row blocks per workgroup
  int32_t wide;            // bf16: two workgroups per 512-column tile, half the rows each
  uint64_t seed;
  void* part;              // [n_slabs][b_max][ell_pad] float (double for F64)
  double* normpart;        // [n_slabs][b_max]
  double* S;               // reduce: l x n_max sketch
  double* colsq;           // reduce: ||a_j||^2 by global column
  int32_t* nonfinite;      // reduce: set when a column norm is not finite
};

// The updates enqueued by one flush share one launch of the SS^T kernel and
// of the tridiagonalisation (one workgroup per update): SS^T and F of update
// u depend only on the sketch, not on the selection.
struct BatchArgs {
  int ell, k, t, nz;
  int64_t u0;             // first update of the batch
  int64_t c0;             // first buffered column of update u0
  int64_t total;          // columns covered by the batch's updates
  double ridge_floor;
  const double* S;
  const double* colsq;
  const double* sst_in;   // SS^T after update u0 - 1
  double* sst_out;        // SS^T after the batch's last update
  double* sst_keep;       // nz slots of l x l: a copy of each update's SS^T (read by Alg. 8)
  double* W;              // nz slots of l x l
  double* hv;             // nz slots of 6 l
  double* Fu;             // ||A_obs||^2 per update
  double* tru;            // tr(SS^T) per update
  int32_t* skipu;         // 1 when the update skips selection (F == 0)
  rid_update* recs;
};

// The split Grams of a run of consecutive updates of a flush in one pass:
// the list holds the columns new at each update of the run, the latest
// update's first, then the others occupied at the run's first update.  Per
// update of the run, the list rows new at it and each list column's slot at
// it (-1 outside its basis).
constexpr int kGramRunMax = 8;      // updates per run
constexpr int kGramRunCols = 256;   // longest list (the 256-column staging)
constexpr int kGramRunTiles = 16;   // 32 x 32 tiles of one split-Gram workgroup
struct GramRun {
  int32_t nq, nj, nu, pad;          // list rows (new columns), list length, updates
  int32_t q0[kGramRunMax], q1[kGramRunMax];
  uint64_t ptr[kGramRunCols];
  int32_t slot[kGramRunMax][kGramRunCols];
};

struct UpdArgs {
  int ell, k, t, n1, n2;
  int64_t u;           // update index
  int64_t c0;          // first column of the buffer
  int cnt;             // buffered columns
  int64_t n_obs;       // observed columns after the buffer
  double fill_mult;    // c (k ln k + k ln(1/delta)/eps) / t
  double ridge_floor;
  uint64_t select_seed;
  int64_t m, ldc;      // rows and column-pool stride
  int data_f64;
  int gram_split;      // binary32 data: Gram on the bfloat16 matrix cores (split form)
  // state
  const double* SSTu;  // SS^T of this update (l x l)
  double* S;           // l x n_max
  double* colsq;
  double* W;           // this update's l x l slot: reflectors below the subdiagonal
  double* hv;          // this update's slot: tau (l), d (l), e (l), Dinv (l), L (l), top eigenvalues (l)
  double* Qs;          // this update's slot: l x l orthogonal factor of the tridiagonalisation
  double* Ys;          // this update's slot: l x (t + cnt) rotated sketch columns of the score items
  double* Fu;          // ||A_obs||^2 per update
  int32_t* skipu;      // 1 when the update skips selection (F == 0)
  int64_t* J;          // t
  double* tau_old;     // t
  double* tauC;        // t (running update)
  double* tauD;        // kMaxT (running update)
  int64_t* J_hist;     // [update][t]
  double* tauC_hist;   // [update][t]
  double* tauD_hist;   // [update][t]
  const uint64_t* colptr;
  void* cpool;         // m x t columns, stride ldc
  uint64_t* slot_ptr;  // t: address of each slot's column (its pool column, or for the split
                       // Gram a snapshot of the running flush not yet copied to the pool)
  int flush_last;      // 1 for the last update of a flush: the split Gram copies the basis
                       // columns still outside the pool
  double* G;           // t x t
  double* gpart;       // gram partials: [slab][gld][gld]
  int gld;             // their leading dimension: t, or 256 when runs of updates share a Gram
  const GramRun* grun; // explicit column list of the split Gram (null: the selection state's)
  int grun_u;          // with grun: the update of the run whose entries the reduction writes
  int gslabs;
  int64_t gslab_rows;
  double* QR;          // l x t
  double* qr_tau;      // t
  double* P;           // t x n_max
  double* Qm;          // l x t: thin Q of Omega A_J (Alg. 4 as products)
  double* Mm;          // t x l: R'^{-1} Q^T
  double* Y;           // l x t  (S P^T)
  double* PPt;         // t x t
  double* hw;          // NA-Hutch++ work
  DevScalars* sc;
  rid_update* recs;
};

// ---------------------------------------------------------------------------
// Batched launches over several streams.
//
// A kernel body takes its arguments by reference and its block coordinates
// as a Blk.  The single-stream kernel passes its own launch's coordinates;
// the batched kernel runs on a grid (max blocks over the streams, streams)
// and block (x, y) decodes x into the coordinates of stream y's own grid,
// whose arguments and grid sit in device tables.  Blocks past a stream's own
// grid exit at once.
// ---------------------------------------------------------------------------
struct Blk {
  int x, y, z;
};
__device__ __forceinline__ Blk own_block() {
  return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
}

template <typename A>
struct Batched {
  const A* args;     // [streams]
  const int4* dims;  // [streams]: grid x, y, z of each stream's own launch
};

template <typename A>
__device__ __forceinline__ bool batched_block(const Batched<A>& L, const A*& a, Blk& bk) {
  const int4 d = L.dims[blockIdx.y];
  int r = (int)blockIdx.x;
  if (r >= d.x * d.y * d.z) return false;
  bk.x = r % d.x;
  r /= d.x;
  bk.y = r % d.y;
  bk.z = r / d.y;
  a = L.args + blockIdx.y;
  return true;
}

// Persistent sketch over several streams: work item q (0 <= q < total) is
// item q - start[s] of stream s, start[] holding the prefix sums of the
// streams' items (n_slabs * n_mt * n_nt); within a stream mt runs fastest,
// then nt, then the slab.
struct MultiSketch {
  const SketchArgs* args;  // [ns]
  const int* start;        // [ns + 1]
  int ns, total;
};

__device__ __forceinline__ void multi_item(const MultiSketch& ms, int q, const SketchArgs*& a, int& slab,
                                           int& mt, int& nt) {
  int lo = 0, hi = ms.ns;  // the last s with start[s] <= q
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ms.start[mid] <= q) lo = mid;
    else hi = mid;
  }
  a = ms.args + lo;
  const int r = q - ms.start[lo];
  mt = r % a->n_mt;
  nt = (r / a->n_mt) % a->n_nt;
  slab = r / (a->n_mt * a->n_nt);
}

// Host side of batched launches: the argument and grid tables of a round are
// written into pinned host memory (`host`), copied to the device mirror
// (`dev`) in one transfer, and the launches reference the device copies.
struct Stage {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0, used = 0;
  bool overflow = false;
  // copies n items to the stage; returns their device address
  template <typename T>
  const T* put(const T* src, size_t n) {
    const size_t at = (used + 255) / 256 * 256;
    if (at + n * sizeof(T) > cap) {
      overflow = true;
      return nullptr;
    }
    memcpy(host + at, src, n * sizeof(T));
    used = at + n * sizeof(T);
    return reinterpret_cast<const T*>(dev + at);
  }
};

// One batched launch, ready to go once the stage has been copied.
struct BLaunch {
  const void* func;
  dim3 grid, block;
  size_t lds;
  const void* args;  // device table (Batched::args, MultiSketch::args)
  const void* aux;   // Batched::dims or MultiSketch::start
  int ns, total;     // MultiSketch only
  int extra;         // trailing int argument (hutch_mid_kernel stage), -1 if none
  bool multi;        // MultiSketch (else Batched)
  int kind;          // for timing: 0 sketch, 1 reduce, 2 update, 3 Gram
  double bytes;      // sketch: snapshot bytes the launch reads
};
hipError_t run_launches(const std::vector<BLaunch>& v, hipStream_t s);

// planners of the batched launches (sketch.hip, update.hip); the host
// argument arrays hold one entry per stream taking part
void plan_sketch_multi(int prec, const SketchArgs* h, int ns, int grid_cap, Stage& st, std::vector<BLaunch>& out);
void plan_sketch_reduce_b(int prec, const SketchArgs* h, int ns, Stage& st, std::vector<BLaunch>& out);
void plan_update_batch_b(const BatchArgs* h, int ns, Stage& st, std::vector<BLaunch>& out);
void plan_update_select_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out, bool with_q = true);
// Q of the tridiagonalisation of each listed update (any mix of streams and updates)
void plan_update_q_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out);
void plan_update_gram_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out);
// want_p[i]: entry i forms P (null: every entry)
void plan_update_coeff_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out,
                         const bool* want_p = nullptr);
// snapshot of the selection state an update's coefficient phase reads
struct SnapArgs {
  const DevScalars* sc;  // state after the update's selection and Gram
  const double* G;
  DevScalars* sc_out;    // the update's snapshot slots
  double* g_out;
  int t;
};
void plan_update_snapshot_b(const SnapArgs* h, int n, Stage& st, std::vector<BLaunch>& out);

// launchers (sketch.hip, update.hip)
// Records the message of a failed call that has no handle and returns st.
rid_status rid_set_global_error(rid_status st, const std::string& msg);

// Rows of the padded test matrix, test-matrix row tiles and 32-row blocks per
// wave of the sketch form `prec` (wide: the bf16 split of a 512-column tile
// over two workgroups).
void sketch_tile_geometry(int prec, int ell, int wide, int* ell_pad, int* n_mt, int* rbw);
// Largest slab (rows summed by one workgroup) of the sketch form `prec`.
int64_t sketch_slab_cap(int prec);
int sketch_cols_per_wg(int prec, int wide);
hipError_t launch_sketch(int prec, const SketchArgs& a, hipStream_t s);
hipError_t launch_sketch_reduce(int prec, const SketchArgs& a, hipStream_t s);
hipError_t launch_omega_block(int prec, uint64_t seed, int ell, int64_t i0, int64_t count,
                              void* out, int64_t ld, hipStream_t s);
hipError_t launch_update_batch(const BatchArgs& b, hipStream_t s);
// Alg. 4 forms P = M S (t x n_obs) through M = R'^{-1} Q^T when t is at most
// this; above it P is formed column by column and Alg. 8 reads P.
constexpr int kAlg4Gemm = 154;
// scores and selection of one update; with_q = false when its Q has been
// formed by launch_update_q_all
hipError_t launch_update_select(const UpdArgs& a, hipStream_t s, bool with_q = true);
// the orthogonal factor Q of the tridiagonalisation of updates a0.u .. a0.u + nz - 1
hipError_t launch_update_q_all(const UpdArgs& a0, int nz, hipStream_t s);
hipError_t launch_update_gram(const UpdArgs& a, hipStream_t s);
// The split Gram of the run of updates a.u - nu + 1 .. a.u (all selected;
// their states in sc_hist / J_hist, a the last one's arguments), a list of
// nq new columns and nj in all (one workgroup's tiles when nu > 1): builds the
// list in run and runs the Gram kernel.  launch_update_gram_run_entries then
// writes update w's entries (w = index in the run; aw its arguments with sc
// and J from the history) and moves its slots' addresses.  Not for the last
// update of a flush.
hipError_t launch_update_gram_run(const UpdArgs& a, int nu, int nq, int nj, const DevScalars* sc_hist,
                                  const int64_t* J_hist, GramRun* run, hipStream_t s);
hipError_t launch_update_gram_run_entries(const UpdArgs& aw, int w, const GramRun* run, hipStream_t s);
// want_p: form P (the last update of a flush; Alg. 8 needs only Y and P P^T)
hipError_t launch_update_coeff(const UpdArgs& a, hipStream_t s, bool want_p = true);
hipError_t launch_update_snapshot(const UpdArgs& a, DevScalars* sc_out, double* g_out, hipStream_t s);

// Algs. 5-7 and the best of four (Alg. 3's coefficient steps).  Buffers of one
// update; layouts as in UpdArgs (column-major, slot-indexed rows of t).
struct B4Args {
  int64_t n_prev;          // columns the previous update's P covers (0 at the first update)
  const int64_t* J_prev;   // t: J of the previous update (null at the first)
  const double* G_prev;    // t x t: basis Gram of the previous update
  double* Xc;              // t x t: products of this update's new columns with the pruned ones
  double* Pc;              // 4 slices of t x n_max: the candidates of Algs. 4, 5, 6, 7
  double* Pprev;           // t x n_max: the previous update's kept P
  double* Pout;            // t x n_max: the stream's P (read by rid_coefficients)
  double* M5;              // t x l: G^{-1} (Omega A_J)^T / l over the occupied slots (Mm layout)
  double* L;               // t x t: Cholesky factor of G over the occupied slots (compact)
  double* T;               // t x t: the Alg. 7 transform (compact current x compact previous slots)
  double* rA;              // l x n_max: the Alg. 6 residual
  double* D6;              // t x n_max: the Alg. 6 correction (rows of the new slots)
  double *QR6, *tau6, *Qm6, *Mm6;  // Alg. 4 factors of the new slots alone
  DevScalars* sc6;         // the selection state restricted to the new slots
  rid_update* scratch_rec; // record the factorisation of the new slots may flag
  rid_update* recq;        // 4: this update's record with each candidate's estimate
  int32_t* qstar;          // this update's kept algorithm (4..7)
  int64_t n_max;
};
// Main stream, between the selection and the Gram of update u >= 1: the
// products of the new basis columns with the pruned ones (before the pool
// copy overwrites the pruned columns).
hipError_t launch_best4_cross(const UpdArgs& a, const B4Args& b, hipStream_t s);
// Second stream, after launch_update_coeff(a with P = Pc slice 0): the other
// three candidates, their estimates and the choice.
hipError_t launch_best4(const UpdArgs& a, const B4Args& b, hipStream_t s);
// NA-Hutch++ work per update (doubles) for l and t; hutch_work_quarter(l) is
// the size of each of its five l^2 / 4 regions
__host__ __device__ inline int64_t hutch_work_quarter(int ell) { return (int64_t)ell * ell / 4 + 64; }
size_t hutch_work_doubles(int ell, int t);

}  // namespace rid
