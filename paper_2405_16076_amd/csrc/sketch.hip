// Sketch contraction S(:, batch) = Omega * A(:, batch) and the column norms
// ||a_j||^2 (eq. random_sketch; Alg. 3 steps 10 and 13).
//
// The contraction is K-dominant (M = l test-matrix rows, N = batch columns,
// K = m snapshot rows).  Rows are split into fixed slabs; one workgroup owns
// (slab, 64 test-matrix rows, a block of columns) and writes an l x b partial
// of that slab; sketch_reduce sums the slabs in a fixed order in binary64.
// The accumulation order of every output element depends only on m and the
// slab size, never on which other columns share the batch, so a column's
// sketch is bitwise the same however the stream is batched.
//
// Omega is never stored: each workgroup regenerates its 64 x KC tile of the
// test matrix per row chunk from the Philox counter (data row, row group) into
// LDS, and every wave of the workgroup multiplies it with its own columns.
#include "rid_internal.h"

#include <algorithm>

namespace rid {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));


// Work item of workgroup `bid`.  Workgroups are dispatched round-robin over the
// eight XCDs; consecutive work items (the tiles of one slab) are given to
// workgroups of the same XCD so that their shared rows meet in its L2.
__device__ __forceinline__ bool sketch_item(const SketchArgs& a, int bid, int& slab, int& mt,
                                            int& nt) {
  const int n_items = a.n_slabs * a.n_mt * a.n_nt;
  const int per_xcd = (n_items + 7) / 8;
  const int q = (bid & 7) * per_xcd + (bid >> 3);
  if (q >= n_items) return false;
  mt = q % a.n_mt;
  nt = (q / a.n_mt) % a.n_nt;
  slab = q / (a.n_mt * a.n_nt);
  return true;
}

// ---------------------------------------------------------------------------
// bfloat16 form: v_mfma_f32_32x32x16_bf16.
// A (32 x 16) lane l holds row l%32, k = 8(l/32)..+8; B (16 x 32) lane l holds
// column l%32, the same k; D lane l holds column l%32, rows
// (v%4) + 4(l/32) + 8(v/4) for v = 0..15.
//
// A workgroup of 8 waves owns (slab, 64*RBW test-matrix rows, 256 columns),
// so every snapshot element is read from HBM by exactly one workgroup.  Wave w
// owns row group w/4 (RBW blocks of 32 rows) and the column pair w%4 (two
// blocks of 32 columns): 2*RBW accumulator tiles; each SIMD (waves s, s+4)
// holds one wave of each row group.  Per 64-row chunk:
//   * the binary32 chunk is copied HBM -> LDS by the LDS-DMA path
//     (global_load_lds_dwordx4) in two halves of 128 columns (32 KB each);
//     every instruction reads whole 256-byte column runs (16 lanes per column,
//     4 columns), and both halves of the next chunk are in flight while one
//     chunk is multiplied;
//   * once a half has landed every thread rounds its part of it to bfloat16
//     into the chunk's bfloat16 stage (32 KB), adding the binary64 column
//     norms, and the half's buffer is refilled with the following chunk at
//     once;
//   * the 64*RBW x 32 tiles of Omega are generated into LDS (double buffered)
//     one half-chunk ahead, each entry one lookup of its Philox half's bits
//     15..5 in a signed copy of the table (entry j: T[j mod 1024] with the
//     sign bit set for j >= 1024).  Row-group-0 waves multiply first and
//     generate second, row-group-1 waves the other way round, so each SIMD
//     overlaps the matrix cores of one wave with the VALU work of the other.
// The products take the k-steps in row order with the same operands for any
// chunking, so every sketch element is the same sum of the same products.
// LDS layouts: a DMA half holds column c at 256*c bytes, lane q of the
// column's 16 fetching lanes at 16*q bytes holding rows 4(q ^ (c % 4))..+4
// (so that the converting reads fall on distinct banks); the bfloat16 stage
// holds column c at 128*c bytes, its 16-byte slot j (rows 8j..8j+7) at
// position j ^ ((c >> 1) & 7).
// ---------------------------------------------------------------------------
constexpr int kBf16Cols = 256;
constexpr int kBf16KC = 64;              // data rows per chunk (256-byte runs)
constexpr int kBf16HC = 32;              // data rows per Omega tile

__device__ __forceinline__ int bf16_slot(int c, int j) { return j ^ ((c >> 1) & 7); }

template <int RBW>
__device__ __forceinline__ void sketch_bf16_body(const SketchArgs& a, int slab, int mt, int nt) {
  constexpr int KC = kBf16KC, HC = kBf16HC;
  constexpr int MROWS = 64 * RBW;        // test-matrix rows per workgroup
  constexpr int LDA = HC + 8;            // bf16 per Omega LDS row (80 bytes)
  // the largest alignment places the signed table at LDS address 0, so a
  // lookup's address is the index doubled, with no base to add
  __shared__ __attribute__((aligned(4096))) uint16_t otab[2 * kOmegaTabSize];
  __shared__ __attribute__((aligned(16))) uint16_t om[2][MROWS * LDA];
  __shared__ __attribute__((aligned(1024))) float stg[2][(kBf16Cols / 2) * KC];
  __shared__ __attribute__((aligned(16))) uint16_t db[kBf16Cols * KC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int rg = wave >> 2, cp = wave & 3;
  load_omega_table_bf16_signed(otab);
  __syncthreads();
  const int64_t r0 = (int64_t)slab * a.slab_rows;
  const int64_t r1 = min(a.m, r0 + a.slab_rows);
  const int nch = (int)((r1 - r0 + KC - 1) / KC);
  const bool ragged = (r1 - r0) % KC != 0;
  const int row_base = mt * MROWS;       // first test-matrix row of this workgroup

  // LDS-DMA geometry: instruction i of wave w for half h copies local columns
  // 128 h + 16 w + 4 i + lane / 16; lane q = lane % 16 of a column fetches the
  // column's rows 4 dq .. 4 dq + 3, dq = q ^ (column % 4).  Columns beyond the
  // batch copy the tile's first column instead: their results are never
  // stored.
  const int dq = (lane & 15) ^ ((lane >> 4) & 3);
  const gmem_t<float>* dsrc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int cl = 128 * h + 16 * wave + 4 * i + (lane >> 4);
      const int cg = nt * kBf16Cols + cl;
      const int cs = cg < a.b ? cg : nt * kBf16Cols;
      dsrc[h][i] = gload_ptr(reinterpret_cast<const float*>(a.colptr[a.c0 + cs]));
    }
  // Rows wholly past the slab end are fetched from row r0 (in bounds) and
  // zeroed when converted; a 16-byte run that straddles the end of the
  // snapshot stays inside the 16-byte-aligned block holding its last row.
  auto issue = [&](int c, int h) {
    int64_t row = r0 + (int64_t)c * KC + 4 * dq;
    if (row >= r1) row = r0;
    const uint32_t sb = lds_addr(&stg[h][0]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      lds_dma16(dsrc[h][i] + row, __builtin_amdgcn_readfirstlane(sb + (uint32_t)(4 * wave + i) * 1024u));
  };

  // Conversion of half h of chunk c: thread t takes rows 16 g .. 16 g + 15
  // (g = t % 4) of the half's column t / 4, adds their squares to the column's
  // norm (binary64, row order) and writes them as two bfloat16 slots.
  double nrm[2] = {0.0, 0.0};
  const int ccl = tid >> 2, g4 = tid & 3;
  auto convert = [&](int c, int h, bool fix) {
    const float* col = &stg[h][ccl * KC];
    const int key = ccl & 3;
    float4 x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = *reinterpret_cast<const float4*>(col + 4 * ((4 * g4 + i) ^ key));
    if (fix) {
      const int64_t k0 = r0 + (int64_t)c * KC + 16 * g4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (k0 + 4 * i >= r1) x[i].x = 0.0f;
        if (k0 + 4 * i + 1 >= r1) x[i].y = 0.0f;
        if (k0 + 4 * i + 2 >= r1) x[i].z = 0.0f;
        if (k0 + 4 * i + 3 >= r1) x[i].w = 0.0f;
      }
    }
    if (mt == 0) {
      double t = nrm[h];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        t = fma((double)x[i].x, (double)x[i].x, t);
        t = fma((double)x[i].y, (double)x[i].y, t);
        t = fma((double)x[i].z, (double)x[i].z, t);
        t = fma((double)x[i].w, (double)x[i].w, t);
      }
      nrm[h] = t;
    }
    const int gc = 128 * h + ccl;
    const bf16x8 lo = bf16x8{(__bf16)x[0].x, (__bf16)x[0].y, (__bf16)x[0].z, (__bf16)x[0].w,
                             (__bf16)x[1].x, (__bf16)x[1].y, (__bf16)x[1].z, (__bf16)x[1].w};
    const bf16x8 hi = bf16x8{(__bf16)x[2].x, (__bf16)x[2].y, (__bf16)x[2].z, (__bf16)x[2].w,
                             (__bf16)x[3].x, (__bf16)x[3].y, (__bf16)x[3].z, (__bf16)x[3].w};
    *reinterpret_cast<u16x8*>(db + gc * KC + 8 * bf16_slot(gc, 2 * g4)) = __builtin_bit_cast(u16x8, lo);
    *reinterpret_cast<u16x8*>(db + gc * KC + 8 * bf16_slot(gc, 2 * g4 + 1)) = __builtin_bit_cast(u16x8, hi);
  };
  // Chunk c into the bfloat16 stage: both its halves are in flight on entry
  // (four copies each per wave, half 0 issued first); each half is refilled
  // with chunk c + 1 as soon as every thread has read it.
  auto convert_chunk = [&](int c) {
    const bool fix = ragged && c == nch - 1;
    wait_dma_keep4();                    // this wave's half-0 copies have landed
    lds_barrier();                       // everyone's; the stage is no longer read
    convert(c, 0, fix);
    wait_dma_all();                      // this wave's half-1 copies have landed
    lds_barrier();                       // everyone's; half 0 has been read
    if (c + 1 < nch) issue(c + 1, 0);
    convert(c, 1, fix);
    lds_barrier();                       // half 1 has been read; the stage is complete
    if (c + 1 < nch) issue(c + 1, 1);
  };

  // Gaussian tile: item = (row group g of 8 rows, data row k of the tile).
  // Row groups at or beyond ell stay zero (written once below).  With 38 row
  // groups the 1216 single Philox calls of a tile fall on the four SIMDs as
  // 5, 5, 5, 4 wave-calls.
  const int n_groups = min(MROWS / 8, max(0, (a.ell - row_base + 7) / 8));
  const int n_items = n_groups * HC;
  auto gen = [&](int64_t k0, uint16_t* d) {
    for (int it = tid; it < n_items; it += 512) {
      const int g = it / HC, k = it % HC;
      uint16_t* dst = d + (8 * g) * LDA + k;
      const Words4 w = omega_words(a.seed, (uint64_t)(k0 + k), (uint32_t)(row_base / 8 + g));
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j * LDA] = otab[(omega_half(w, j) >> 5) & (2 * kOmegaTabSize - 1)];
    }
  };

  f32x16 acc[RBW][2];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.0f;

  // Half hh of the chunk on the matrix cores: k-steps s = 2 hh, 2 hh + 1
  // (rows 16 s .. 16 s + 15) against the Omega tile O of those 32 rows; lane
  // (l32, half) reads rows 16 s + 8 half .. +8 of column (2 cp + cc) 32 + l32.
  auto mfma_half = [&](const uint16_t* O, int hh) {
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int s = 2 * hh + s2;
      bf16x8 bop[2];
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int cl = (2 * cp + cc) * 32 + l32;
        bop[cc] = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const u16x8*>(db + cl * KC + 8 * bf16_slot(cl, 2 * s + half)));
      }
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
        const bf16x8 av = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const u16x8*>(&O[((rg * RBW + r) * 32 + l32) * LDA + 16 * s2 + 8 * half]));
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
          acc[r][cc] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bop[cc], acc[r][cc], 0, 0, 0);
      }
    }
  };

  // prologue: both halves of chunk 0 in flight, zero rows of Omega, the Omega
  // tile of rows 0..31, chunk 0 converted (chunk 1 then in flight)
  issue(0, 0);
  issue(0, 1);
  for (int i = tid + n_groups * 8 * (LDA / 2); i < MROWS * (LDA / 2); i += 512) {
    reinterpret_cast<uint32_t*>(om[0])[i] = 0u;
    reinterpret_cast<uint32_t*>(om[1])[i] = 0u;
  }
  gen(r0, om[0]);
  convert_chunk(0);

  for (int c = 0; c < nch; ++c) {
    const int64_t kb = r0 + (int64_t)c * KC;
    const bool more = c + 1 < nch;
    // rows 0..31 against om[0]; the tile of rows 32..63 into om[1]
    if (rg == 0) {
      mfma_half(om[0], 0);
      gen(kb + HC, om[1]);
    } else {
      gen(kb + HC, om[1]);
      mfma_half(om[0], 0);
    }
    lds_barrier();
    // rows 32..63 against om[1]; the next chunk's rows 0..31 into om[0]
    if (rg == 0) {
      mfma_half(om[1], 1);
      if (more) gen(kb + KC, om[0]);
    } else {
      if (more) gen(kb + KC, om[0]);
      mfma_half(om[1], 1);
    }
    if (more) convert_chunk(c + 1);
  }

  float* part = reinterpret_cast<float*>(a.part);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = nt * kBf16Cols + (2 * cp + c) * 32 + l32;
    if (col >= a.b) continue;
    float* dst = part + ((int64_t)slab * a.b_max + col) * a.ell_pad + row_base;
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float4 v = make_float4(acc[r][c][4 * q], acc[r][c][4 * q + 1], acc[r][c][4 * q + 2],
                               acc[r][c][4 * q + 3]);
        *reinterpret_cast<float4*>(dst + (rg * RBW + r) * 32 + 8 * q + 4 * half) = v;
      }
  }
  if (mt == 0) {
    // the four threads of a column add their sums with a fixed butterfly
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double t = nrm[h];
      t += __shfl_xor(t, 1);
      t += __shfl_xor(t, 2);
      const int col = nt * kBf16Cols + 128 * h + ccl;
      if (g4 == 0 && col < a.b) a.normpart[(int64_t)slab * a.b_max + col] = t;
    }
  }
}

template <int RBW>
__global__ __launch_bounds__(512, 1) void sketch_bf16_kernel(SketchArgs a) {
  int slab, mt, nt;
  if (sketch_item(a, blockIdx.x, slab, mt, nt)) sketch_bf16_body<RBW>(a, slab, mt, nt);
}

template <int RBW>
__global__ __launch_bounds__(512, 1) void sketch_bf16_multi(MultiSketch ms) {
  int slab, mt, nt;
  const SketchArgs* a;
  for (int q = blockIdx.x; q < ms.total; q += gridDim.x) {
    multi_item(ms, q, a, slab, mt, nt);
    sketch_bf16_body<RBW>(*a, slab, mt, nt);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Wide bfloat16 form: two workgroups share a 512-column tile, each taking
// half of the sketch rows (32 RB rows), so each Gaussian of a tile row is
// generated for 512 columns instead of 256; the two workgroups of a tile are
// consecutive work items (same XCD, started together), so the columns one
// of them fetches from HBM meet the other in L2.  Wave w owns column blocks
// 2w, 2w+1 and every row block: RB x 2 accumulator tiles, as in the narrow
// form.  Chunks of 32 rows x 512 columns (64 KB) go HBM -> LDS by LDS-DMA
// into two stages (one chunk in flight while one is consumed); the Omega
// tile of the next chunk is generated during the current one (waves 0-3
// multiply first, waves 4-7 generate first).  Items of the generation are
// single Philox calls (8 rows x 1 data row) spread over all 512 threads.
// ---------------------------------------------------------------------------
constexpr int kWideCols = 512;

template <int RB>
__device__ __forceinline__ void sketch_bf16w_body(const SketchArgs& a, int slab, int mt, int nt) {
  constexpr int KC = 32;                 // rows per chunk
  constexpr int MROWS = 32 * RB;         // test-matrix rows per workgroup
  constexpr int LDA = KC + 8;            // bf16 per Omega LDS row (80 bytes)
  __shared__ __attribute__((aligned(16))) uint16_t om[2][MROWS * LDA];
  __shared__ __attribute__((aligned(1024))) float dt[2][kWideCols * KC];
  __shared__ uint64_t csrc[kWideCols];
  __shared__ __attribute__((aligned(16))) uint16_t otab[kOmegaTabSize];
  load_omega_table(otab, kOmegaTabBf16);
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int64_t r0 = (int64_t)slab * a.slab_rows;
  const int64_t r1 = min(a.m, r0 + a.slab_rows);
  const int nch = (int)((r1 - r0 + KC - 1) / KC);
  const bool ragged = (r1 - r0) % KC != 0;
  const int row_base = mt * MROWS;

  // column addresses (columns past the batch read the tile's first column;
  // their results are never stored)
  for (int cl = tid; cl < kWideCols; cl += 512) {
    const int cg = nt * kWideCols + cl;
    csrc[cl] = a.colptr[a.c0 + (cg < a.b ? cg : nt * kWideCols)];
  }
  __syncthreads();
  // LDS-DMA: copy i of wave w fills columns 8(8w+i)..+8 of a chunk, 8 lanes
  // per column; rows wholly past the slab end come from row r0 and are zeroed
  // by the fix-up, a run straddling the snapshot end stays in its 16-byte block
  auto issue = [&](int c) {
    const int64_t k0 = r0 + (int64_t)c * KC;
    const uint32_t sb = lds_addr(&dt[c & 1][0]);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int cl = 8 * (8 * wave + i) + (lane >> 3);
      int64_t row = k0 + 4 * ((lane & 7) ^ col_swz(cl));
      if (row >= r1) row = r0;
      const gmem_t<float>* src = gload_ptr(reinterpret_cast<const float*>(csrc[cl]));
      lds_dma16(src + row, __builtin_amdgcn_readfirstlane(sb + (uint32_t)(8 * wave + i) * 1024u));
    }
  };
  auto fixup = [&](int c) {
    const int64_t k0 = r0 + (int64_t)c * KC;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int cl = 8 * (8 * wave + i) + (lane >> 3);
      const int64_t row = k0 + 4 * ((lane & 7) ^ col_swz(cl));
      float* slot = &dt[c & 1][cl * KC + 4 * (lane & 7)];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (row + e >= r1) slot[e] = 0.0f;
    }
  };

  // Omega tile of chunk c: item = (row group g, data row k), one Philox call
  const int n_groups = min(MROWS / 8, max(0, (a.ell - row_base + 7) / 8));
  const int n_items = n_groups * KC;
  auto gen = [&](int c) {
    const int64_t k0 = r0 + (int64_t)c * KC;
    uint16_t* d = om[c & 1];
    for (int it = tid; it < n_items; it += 512) {
      const int g = it / KC, k = it % KC;
      uint16_t z[8];
      omega8_bf16(a.seed, (uint64_t)(k0 + k), (uint32_t)(row_base / 8 + g), otab, z);
#pragma unroll
      for (int j = 0; j < 8; ++j) d[(8 * g + j) * LDA + k] = z[j];
    }
  };

  f32x16 acc[RB][2];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.0f;
  double nrm[2] = {0.0, 0.0};

  // one chunk on the matrix cores; lane (l32, half) reads rows
  // 16 s + 8 half .. +8 of column (2 wave + cc) 32 + l32 (each element once,
  // which also gives the binary64 norms)
  auto mfma_chunk = [&](int c) {
    const uint16_t* O = om[c & 1];
    const float* D = dt[c & 1];
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      bf16x8 bop[2];
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int cl = (2 * wave + cc) * 32 + l32;
        const int key = col_swz(cl);
        const float* colb = D + cl * KC;
        const float4 x0 = *reinterpret_cast<const float4*>(colb + 4 * ((4 * s + 2 * half) ^ key));
        const float4 x1 = *reinterpret_cast<const float4*>(colb + 4 * ((4 * s + 2 * half + 1) ^ key));
        if (mt == 0) {
          double t = nrm[cc];
          t = fma((double)x0.x, (double)x0.x, t);
          t = fma((double)x0.y, (double)x0.y, t);
          t = fma((double)x0.z, (double)x0.z, t);
          t = fma((double)x0.w, (double)x0.w, t);
          t = fma((double)x1.x, (double)x1.x, t);
          t = fma((double)x1.y, (double)x1.y, t);
          t = fma((double)x1.z, (double)x1.z, t);
          t = fma((double)x1.w, (double)x1.w, t);
          nrm[cc] = t;
        }
        bop[cc] = bf16x8{(__bf16)x0.x, (__bf16)x0.y, (__bf16)x0.z, (__bf16)x0.w,
                         (__bf16)x1.x, (__bf16)x1.y, (__bf16)x1.z, (__bf16)x1.w};
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const bf16x8 av = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const u16x8*>(&O[(r * 32 + l32) * LDA + 16 * s + 8 * half]));
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
          acc[r][cc] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bop[cc], acc[r][cc], 0, 0, 0);
      }
    }
  };

  // prologue: chunk 0 in flight, zero rows of Omega, Omega of chunk 0
  issue(0);
  for (int i = tid + n_groups * 8 * (LDA / 2); i < MROWS * (LDA / 2); i += 512) {
    reinterpret_cast<uint32_t*>(om[0])[i] = 0u;
    reinterpret_cast<uint32_t*>(om[1])[i] = 0u;
  }
  gen(0);
  wait_dma_all();
  if (ragged && nch == 1) fixup(0);
  lds_barrier();
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) issue(c + 1);       // the stage of chunk c - 1 is free
    if (wave < 4) {
      mfma_chunk(c);
      if (c + 1 < nch) gen(c + 1);
    } else {
      if (c + 1 < nch) gen(c + 1);
      mfma_chunk(c);
    }
    wait_dma_all();
    if (ragged && c + 1 == nch - 1) fixup(c + 1);
    lds_barrier();
  }

  float* part = reinterpret_cast<float*>(a.part);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = nt * kWideCols + (2 * wave + c) * 32 + l32;
    if (col >= a.b) continue;
    float* dst = part + ((int64_t)slab * a.b_max + col) * a.ell_pad + row_base;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float4 v = make_float4(acc[r][c][4 * q], acc[r][c][4 * q + 1], acc[r][c][4 * q + 2],
                               acc[r][c][4 * q + 3]);
        *reinterpret_cast<float4*>(dst + r * 32 + 8 * q + 4 * half) = v;
      }
  }
  if (mt == 0) {
    // lanes l and l + 32 hold the two row halves of one column
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const double t = nrm[cc] + __shfl_xor(nrm[cc], 32);
      const int col = nt * kWideCols + (2 * wave + cc) * 32 + l32;
      if (half == 0 && col < a.b) a.normpart[(int64_t)slab * a.b_max + col] = t;
    }
  }
}

template <int RB>
__global__ __launch_bounds__(512, 1) void sketch_bf16w_kernel(SketchArgs a) {
  int slab, mt, nt;
  if (sketch_item(a, blockIdx.x, slab, mt, nt)) sketch_bf16w_body<RB>(a, slab, mt, nt);
}

template <int RB>
__global__ __launch_bounds__(512, 1) void sketch_bf16w_multi(MultiSketch ms) {
  int slab, mt, nt;
  const SketchArgs* a;
  for (int q = blockIdx.x; q < ms.total; q += gridDim.x) {
    multi_item(ms, q, a, slab, mt, nt);
    sketch_bf16w_body<RB>(*a, slab, mt, nt);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// fp8 form: e4m3 operands with power-of-two block scales on
// v_mfma_scale_f32_32x32x64_f8f6f4 (binary32 accumulation).
//   * Omega is e4m3(Omega * 2^6) with the fixed scale 2^-6 (E8M0 121).
//   * The data carries one scale per 32 rows of each column: 2^(floor(log2
//     max|x|) - 7), so the scaled block maximum lies in [128, 256).
// Operand layout of the instruction (e4m3, 8 VGPRs per lane): lane l holds
// row (A) / column (B) l%32; its bytes 0..15 lie in k-block 0 (k < 32) and
// bytes 16..31 in k-block 1; the E8M0 scale given by lane l applies to row /
// column l%32 within k-block l/32.  Here lane (c, h = l/32) carries rows
// 16h..16h+15 of each 32-row block (bytes 0..15: block 0, bytes 16..31:
// block 1) for both operands, so A and B agree on k.
//
// One workgroup per (slab, 64*RBW sketch rows, 256 columns) as in the bfloat16
// form.  A step consumes 64 data rows = two 32-row chunks (one scale block
// each) of a four-stage LDS-DMA ring, in three phases split by barriers:
//   quantize  thread t takes column t%256 of chunk t/256: it reads the 32
//             binary32 values (zeroing rows past the slab), adds their squares
//             to its binary64 norm, picks the block scale and writes the 32
//             e4m3 codes back over the first 32 bytes of the same column run
//             (16-byte halves at slots swz(c) and swz(c)^4), its E8M0 code to
//             a table;
//   multiply  each wave runs its 2*RBW scaled MFMAs on the quantized step and
//             the Omega tile (64*RBW rows x 64 data rows, 80-byte rows);
//   refill    the two consumed chunks are re-issued four chunks ahead and the
//             next Omega tile is generated.
// Quantizing once per column (not once per consuming wave) keeps the binary32
// values out of the registers of the multiply phase, where the 2*RBW
// accumulator tiles fill the register file.
// ---------------------------------------------------------------------------
typedef int v8i_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int fp8_block_exp(float amax) {
  if (!(amax > 0.0f)) return -127;
  const int e = ilogbf(amax) - 7;  // floor(log2 amax) - 7
  return e < -127 ? -127 : (e > 127 ? 127 : e);
}
__device__ __forceinline__ void wait_dma_keep(int n) {
  if (n >= 8) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
  else if (n >= 4) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

template <int RBW>
__device__ __forceinline__ void sketch_fp8_body(const SketchArgs& a, int slab, int mt, int nt) {
  constexpr int KC = 32;                 // rows per DMA chunk (one scale block)
  constexpr int NST = 4;                 // DMA stages
  constexpr int MROWS = 64 * RBW;        // test-matrix rows per workgroup
  constexpr int LDO = 80;                // bytes per Omega tile row (64 + pad)
  // the signed e4m3 table at LDS address 0 (the largest alignment is placed
  // first), so that a half's bits 15..5 address it with no base add
  __shared__ __attribute__((aligned(2048))) uint8_t otab[2 * kOmegaTabSize];
  __shared__ __attribute__((aligned(16))) uint8_t om[MROWS * LDO];
  __shared__ __attribute__((aligned(1024))) float dt[NST][kBf16Cols * KC];
  __shared__ uint64_t csrc[kBf16Cols];
  __shared__ int scl[2][kBf16Cols];      // E8M0 code of (chunk of the step, column)
  load_omega_table_e4m3_signed(otab);
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int rg = wave >> 2, cp = wave & 3;
  const int64_t r0 = (int64_t)slab * a.slab_rows;
  const int64_t r1 = min(a.m, r0 + a.slab_rows);
  const int nch = (int)((r1 - r0 + KC - 1) / KC);
  const int nsteps = (nch + 1) / 2;
  const int row_base = mt * MROWS;

  for (int cl = tid; cl < kBf16Cols; cl += 512) {
    const int cg = nt * kBf16Cols + cl;
    csrc[cl] = a.colptr[a.c0 + (cg < a.b ? cg : nt * kBf16Cols)];
  }
  __syncthreads();
  // LDS-DMA: copy i of wave w fills columns 8(4w+i)..+8 of a chunk.  Rows
  // wholly past the slab end are fetched from row r0 (in bounds) and zeroed by
  // the quantize phase; a 16-byte run that straddles the end of the snapshot
  // stays inside the 16-byte-aligned block holding its last row.
  auto issue = [&](int c) {
    if (c >= nch) return;
    const int64_t k0 = r0 + (int64_t)c * KC;
    const uint32_t sb = lds_addr(&dt[c % NST][0]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int cl = 8 * (4 * wave + i) + (lane >> 3);
      int64_t row = k0 + 4 * ((lane & 7) ^ col_swz(cl));
      if (row >= r1) row = r0;
      const gmem_t<float>* src = gload_ptr(reinterpret_cast<const float*>(csrc[cl]));
      lds_dma16(src + row, __builtin_amdgcn_readfirstlane(sb + (uint32_t)(4 * wave + i) * 1024u));
    }
  };
  // copies issued after chunk c (they may still be in flight when c is needed)
  auto later = [&](int c) { return max(0, min(nch - 1, c + 2) - c) * 4; };

  // Omega tile of step q: item = (row group g, data rows 2 kp, 2 kp + 1): two
  // Philox calls give 8 x 2 entries, written as one 16-bit word per row.
  // With 38 row groups the 1216 items of a step fall on the four SIMDs as
  // 10, 10, 10, 8 wave-calls (items of four calls gave 12, 12, 8, 8).
  // Row groups at or beyond ell stay zero (written once below).
  const int n_groups = min(MROWS / 8, max(0, (a.ell - row_base + 7) / 8));
  const int n_items = n_groups * 32;
  auto gen = [&](int q) {
    const int64_t k0 = r0 + (int64_t)q * 64;
    for (int it = tid; it < n_items; it += 512) {
      const int g = it >> 5, kp = it & 31;
      const Words4 w0 = omega_words(a.seed, (uint64_t)(k0 + 2 * kp), (uint32_t)(row_base / 8 + g));
      const Words4 w1 = omega_words(a.seed, (uint64_t)(k0 + 2 * kp + 1), (uint32_t)(row_base / 8 + g));
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t z0 = otab[(omega_half(w0, j) >> 5) & (2 * kOmegaTabSize - 1)];
        const uint32_t z1 = otab[(omega_half(w1, j) >> 5) & (2 * kOmegaTabSize - 1)];
        *reinterpret_cast<uint16_t*>(&om[(8 * g + j) * LDO + 2 * kp]) = (uint16_t)(z0 | (z1 << 8));
      }
    }
  };

  // quantize phase of step s (see above); nrm is this thread's column norm
  const int qcl = tid & (kBf16Cols - 1), qcb = tid >> 8;
  const int qswz = col_swz(qcl);
  double nrm = 0.0;
  auto quantize = [&](int s) {
    const int c = 2 * s + qcb;
    float* col = &dt[c % NST][qcl * KC];
    float x[32];
    if (c < nch) {
      const int64_t k0 = r0 + (int64_t)c * KC;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float4 v = *reinterpret_cast<const float4*>(col + 4 * (q ^ qswz));
        x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
      }
      if (k0 + KC > r1) {
#pragma unroll
        for (int q = 0; q < 32; ++q)
          if (k0 + q >= r1) x[q] = 0.0f;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 32; ++q) x[q] = 0.0f;
    }
    double t = nrm;
    float mx = 0.0f;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      t = fma((double)x[q], (double)x[q], t);
      mx = fmaxf(mx, fabsf(x[q]));
    }
    nrm = t;
    const int e = fp8_block_exp(mx);
    const float inv = __builtin_ldexpf(1.0f, -e);
    int w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int v = __builtin_amdgcn_cvt_pk_fp8_f32(x[4 * q] * inv, x[4 * q + 1] * inv, 0, false);
      w[q] = __builtin_amdgcn_cvt_pk_fp8_f32(x[4 * q + 2] * inv, x[4 * q + 3] * inv, v, true);
    }
    *reinterpret_cast<int4*>(col + 4 * qswz) = make_int4(w[0], w[1], w[2], w[3]);
    *reinterpret_cast<int4*>(col + 4 * (qswz ^ 4)) = make_int4(w[4], w[5], w[6], w[7]);
    scl[qcb][qcl] = e + 127;
  };

  f32x16 acc[RBW][2];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.0f;

  // multiply phase of step s: lane (l32, half) supplies rows 16 half..+16 of
  // both chunks of column (2 cp + cc) 32 + l32 and the scale of chunk `half`.
  // The Omega operand of block r + 1 is loaded while block r multiplies; the
  // scheduling fences keep the compiler from hoisting all of them at once.
  auto load_a = [&](int r) {
    const uint8_t* orow = &om[((rg * RBW + r) * 32 + l32) * LDO];
    const int4 lo = *reinterpret_cast<const int4*>(orow + 16 * half);
    const int4 hi = *reinterpret_cast<const int4*>(orow + 32 + 16 * half);
    return v8i_t{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  };
  auto multiply = [&](int s) {
    v8i_t bop[2];
    int bsc[2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const int cl = (2 * cp + cc) * 32 + l32;
      const int slot = col_swz(cl) ^ (4 * half);
      const int4 b0 = *reinterpret_cast<const int4*>(&dt[(2 * s) % NST][cl * KC + 4 * slot]);
      const int4 b1 = *reinterpret_cast<const int4*>(&dt[(2 * s + 1) % NST][cl * KC + 4 * slot]);
      bop[cc] = v8i_t{b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
      bsc[cc] = scl[half][cl];
    }
    v8i_t av = load_a(0);
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      v8i_t an = av;
      if (r + 1 < RBW) an = load_a(r + 1);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc)
        acc[r][cc] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bop[cc], acc[r][cc], 0, 0, 0, 121, 0,
                                                                     bsc[cc]);
      __builtin_amdgcn_sched_barrier(0);
      av = an;
    }
    // keep the products in this phase (not sunk past the barrier, where the
    // operands would stay live across the refill code)
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) asm volatile("" ::"v"(acc[r][cc][0]));
  };

  // prologue: chunks 0..3 in flight, zero rows of Omega, Omega of step 0,
  // quantized step 0
#pragma unroll
  for (int c = 0; c < NST; ++c) issue(c);
  for (int i = tid + n_groups * 8 * (LDO / 4); i < MROWS * (LDO / 4); i += 512)
    reinterpret_cast<int*>(om)[i] = 0;
  gen(0);
  wait_dma_keep(later(1));               // chunks 0 and 1 have landed
  lds_barrier();
  quantize(0);
  lds_barrier();
  for (int s = 0; s < nsteps; ++s) {
    multiply(s);
    lds_barrier();                       // Omega tile and chunks 2s, 2s+1 are free
    issue(2 * s + 4);
    issue(2 * s + 5);
    if (s + 1 < nsteps) gen(s + 1);
    wait_dma_keep(later(2 * s + 3));     // chunks 2s+2, 2s+3 have landed
    lds_barrier();
    if (s + 1 < nsteps) quantize(s + 1);
    lds_barrier();
  }

  float* part = reinterpret_cast<float*>(a.part);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = nt * kBf16Cols + (2 * cp + c) * 32 + l32;
    if (col >= a.b) continue;
    float* dst = part + ((int64_t)slab * a.b_max + col) * a.ell_pad + row_base;
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float4 v = make_float4(acc[r][c][4 * q], acc[r][c][4 * q + 1], acc[r][c][4 * q + 2],
                               acc[r][c][4 * q + 3]);
        *reinterpret_cast<float4*>(dst + (rg * RBW + r) * 32 + 8 * q + 4 * half) = v;
      }
  }
  if (mt == 0) {
    // the two chunk parities of a column meet in LDS (the ring is idle now)
    double* nsh = reinterpret_cast<double*>(&dt[0][0]);
    if (qcb == 1) nsh[qcl] = nrm;
    __syncthreads();
    if (qcb == 0) {
      const int col = nt * kBf16Cols + qcl;
      if (col < a.b) a.normpart[(int64_t)slab * a.b_max + col] = nrm + nsh[qcl];
    }
  }
}

template <int RBW>
__global__ __launch_bounds__(512, 1) void sketch_fp8_kernel(SketchArgs a) {
  int slab, mt, nt;
  if (sketch_item(a, blockIdx.x, slab, mt, nt)) sketch_fp8_body<RBW>(a, slab, mt, nt);
}

template <int RBW>
__global__ __launch_bounds__(512, 1) void sketch_fp8_multi(MultiSketch ms) {
  int slab, mt, nt;
  const SketchArgs* a;
  for (int q = blockIdx.x; q < ms.total; q += gridDim.x) {
    multi_item(ms, q, a, slab, mt, nt);
    sketch_fp8_body<RBW>(*a, slab, mt, nt);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// binary32 form: v_mfma_f32_32x32x2_f32 (A lane l: row l%32, k = l/32; B lane
// l: column l%32, k = l/32).  Within a 16-row chunk lane half h reads rows
// 8h..8h+7 of its column and MFMA step s uses row 8h+s of both operands.
// ---------------------------------------------------------------------------
template <int NCB>
__device__ __forceinline__ void sketch_f32_body(const SketchArgs& a, int slab, int mt, int nt) {
  constexpr int KC = 16;
  constexpr int LD = KC + 4;  // floats per LDS tile row (80 bytes)
  __shared__ __attribute__((aligned(16))) float om[kMTile * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int64_t r0 = (int64_t)slab * a.slab_rows;
  const int64_t r1 = min(a.m, r0 + a.slab_rows);

  const gmem_t<float>* colp[NCB];
  bool ok[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int c = nt * (4 * NCB * 32) + wave * (NCB * 32) + cb * 32 + l32;
    ok[cb] = c < a.b;
    colp[cb] = gload_ptr(ok[cb] ? reinterpret_cast<const float*>(a.colptr[a.c0 + c]) : nullptr);
  }
  f32x16 acc[2][NCB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[rb][cb][v] = 0.0f;
  double nrm[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) nrm[cb] = 0.0;

  const int gk = tid & 15, gg = tid >> 4;  // tid < 128 generate
  for (int64_t k0 = r0; k0 < r1; k0 += KC) {
    if (tid < 128) {
      float z[8];
      omega8_f32(a.seed, (uint64_t)(k0 + gk), (uint32_t)(mt * (kMTile / 8) + gg), z);
#pragma unroll
      for (int j = 0; j < 8; ++j) om[(8 * gg + j) * LD + gk] = z[j];
    }
    __syncthreads();
    float x[NCB][8];
    const int64_t rr = k0 + 8 * half;
    const bool full = (k0 + KC <= r1);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      if (ok[cb] && full) {
        const float4 v0 = gload_f4(colp[cb] + rr), v1 = gload_f4(colp[cb] + rr + 4);
        x[cb][0] = v0.x; x[cb][1] = v0.y; x[cb][2] = v0.z; x[cb][3] = v0.w;
        x[cb][4] = v1.x; x[cb][5] = v1.y; x[cb][6] = v1.z; x[cb][7] = v1.w;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[cb][j] = (ok[cb] && rr + j < r1) ? colp[cb][rr + j] : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) nrm[cb] = fma((double)x[cb][j], (double)x[cb][j], nrm[cb]);
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const float4* ap = reinterpret_cast<const float4*>(&om[(rb * 32 + l32) * LD + 8 * half]);
      const float4 a0 = ap[0], a1 = ap[1];
      const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], x[cb][s], acc[rb][cb], 0, 0, 0);
    }
    __syncthreads();
  }

  float* part = reinterpret_cast<float*>(a.part);
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    if (!ok[cb]) continue;
    const int c = nt * (4 * NCB * 32) + wave * (NCB * 32) + cb * 32 + l32;
    float* dst = part + ((int64_t)slab * a.b_max + c) * a.ell_pad + mt * kMTile;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float4 v = make_float4(acc[rb][cb][4 * q], acc[rb][cb][4 * q + 1], acc[rb][cb][4 * q + 2],
                               acc[rb][cb][4 * q + 3]);
        *reinterpret_cast<float4*>(dst + rb * 32 + 8 * q + 4 * half) = v;
      }
  }
  if (mt == 0) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const double tot = nrm[cb] + __shfl_xor(nrm[cb], 32);
      const int c = nt * (4 * NCB * 32) + wave * (NCB * 32) + cb * 32 + l32;
      if (ok[cb] && half == 0) a.normpart[(int64_t)slab * a.b_max + c] = tot;
    }
  }
}

template <int NCB>
__global__ __launch_bounds__(256) void sketch_f32_kernel(SketchArgs a) {
  int slab, mt, nt;
  if (sketch_item(a, blockIdx.x, slab, mt, nt)) sketch_f32_body<NCB>(a, slab, mt, nt);
}

template <int NCB>
__global__ __launch_bounds__(256) void sketch_f32_multi(MultiSketch ms) {
  int slab, mt, nt;
  const SketchArgs* a;
  for (int q = blockIdx.x; q < ms.total; q += gridDim.x) {
    multi_item(ms, q, a, slab, mt, nt);
    sketch_f32_body<NCB>(*a, slab, mt, nt);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// binary64 form: 64 test-matrix rows x 64 columns per workgroup, 16-row
// chunks staged in LDS, 4 x 4 outputs per thread, binary64 FMA.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sketch_f64_body(const SketchArgs& a, int slab, int mt, int nt) {
  constexpr int KC = 16, NTC = 64;
  __shared__ double om[KC][kMTile + 1];
  __shared__ double dt[KC][NTC + 1];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const int64_t r0 = (int64_t)slab * a.slab_rows;
  const int64_t r1 = min(a.m, r0 + a.slab_rows);
  // data loading: thread -> column lc = tid / 4, rows 4 (tid % 4) .. +4
  const int lc = tid >> 2, lr = (tid & 3) * 4;
  const int cglob = nt * NTC + lc;
  const bool cok = cglob < a.b;
  const gmem_t<double>* cp = gload_ptr(cok ? reinterpret_cast<const double*>(a.colptr[a.c0 + cglob]) : nullptr);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  double nrm = 0.0;
  for (int64_t k0 = r0; k0 < r1; k0 += KC) {
    if (tid < 128) {
      const int gk = tid & 15, gg = tid >> 4;
      double z[8];
      omega8_f64(a.seed, (uint64_t)(k0 + gk), (uint32_t)(mt * (kMTile / 8) + gg), z);
#pragma unroll
      for (int j = 0; j < 8; ++j) om[gk][8 * gg + j] = z[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t row = k0 + lr + j;
      const double v = (cok && row < r1) ? cp[row] : 0.0;
      dt[lr + j][lc] = v;
      nrm = fma(v, v, nrm);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = om[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = dt[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* part = reinterpret_cast<double*>(a.part);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = nt * NTC + tx * 4 + j;
    if (c >= a.b) continue;
    double* dst = part + ((int64_t)slab * a.b_max + c) * a.ell_pad + mt * kMTile + ty * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = acc[i][j];
  }
  if (mt == 0) {
    // the four threads of a column hold disjoint row quarters of every chunk
    nrm += __shfl_xor(nrm, 1);
    nrm += __shfl_xor(nrm, 2);
    if ((tid & 3) == 0 && cok) a.normpart[(int64_t)slab * a.b_max + cglob] = nrm;
  }
}

__global__ __launch_bounds__(256) void sketch_f64_kernel(SketchArgs a) {
  int slab, mt, nt;
  if (sketch_item(a, blockIdx.x, slab, mt, nt)) sketch_f64_body(a, slab, mt, nt);
}

__global__ __launch_bounds__(256) void sketch_f64_multi(MultiSketch ms) {
  int slab, mt, nt;
  const SketchArgs* a;
  for (int q = blockIdx.x; q < ms.total; q += gridDim.x) {
    multi_item(ms, q, a, slab, mt, nt);
    sketch_f64_body(*a, slab, mt, nt);
    __syncthreads();
  }
}

// Fixed-order binary64 sum of the slab partials into S(:, c0:c0+b) and
// ||a_j||^2; a non-finite norm (a non-finite snapshot value) sets the flag.
// Block (x, y): rows 64 x.., column y of the batch.
// One workgroup of NWR waves per (64 sketch rows, column): wave w sums the
// w-th share of the slabs in slab order, then the shares are added in wave
// order.  The column's norm: lane i of wave 1 sums slabs i, i + 64, ..., then a
// fixed butterfly over the lanes, lane 0's result kept.  A single stream's
// hundreds of slabs take 16 waves; a batch's members, most with few slabs,
// take 4.
constexpr int kReduceWaves = 16;
constexpr int kReduceWavesBatch = 4;

template <typename T, int NWR>
__device__ __forceinline__ void sketch_reduce_body(const SketchArgs& a, const Blk bk) {
  __shared__ double share[NWR][64];
  const T* __restrict__ part = reinterpret_cast<const T*>(a.part);
  const int c = bk.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = bk.x * 64 + lane;
  if (c >= a.b) return;  // the same for the whole workgroup
  const int per = (a.n_slabs + NWR - 1) / NWR;
  const int s1 = min(a.n_slabs, (w + 1) * per);
  double s = 0.0;
  if (r < a.ell) {
#pragma unroll 8
    for (int sl = w * per; sl < s1; ++sl) s += (double)part[((int64_t)sl * a.b_max + c) * a.ell_pad + r];
  }
  share[w][lane] = s;
  __syncthreads();
  if (w == 0 && r < a.ell) {
    double tot = share[0][lane];
#pragma unroll
    for (int i = 1; i < NWR; ++i) tot += share[i][lane];
    a.S[(a.c0 + c) * a.ell + r] = tot;
  }
  if (bk.x == 0 && w == 1) {
    double q = 0.0;
    for (int sl = lane; sl < a.n_slabs; sl += 64) q += a.normpart[(int64_t)sl * a.b_max + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
    if (lane == 0) {
      a.colsq[a.c0 + c] = q;
      if (!isfinite(q)) *a.nonfinite = 1;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(64 * kReduceWaves) void sketch_reduce_kernel(SketchArgs a) {
  sketch_reduce_body<T, kReduceWaves>(a, own_block());
}

template <typename T>
__global__ __launch_bounds__(64 * kReduceWavesBatch) void sketch_reduce_kernel_b(Batched<SketchArgs> L) {
  const SketchArgs* a;
  Blk bk;
  if (batched_block(L, a, bk)) sketch_reduce_body<T, kReduceWavesBatch>(*a, bk);
}

__global__ void omega_block_kernel(int prec, uint64_t seed, int ell, int64_t i0, int64_t count,
                                   void* out, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (i >= count) return;
  if (prec == RID_SKETCH_F64) {
    double z[8];
    omega8_f64(seed, (uint64_t)(i0 + i), (uint32_t)g, z);
    for (int j = 0; j < 8; ++j)
      if (8 * g + j < ell) reinterpret_cast<double*>(out)[i * ld + 8 * g + j] = z[j];
  } else {
    float z[8];
    if (prec == RID_SKETCH_F32) {
      omega8_f32(seed, (uint64_t)(i0 + i), (uint32_t)g, z);
    } else if (prec == RID_SKETCH_BF16) {
      uint16_t b[8];
      omega8_bf16(seed, (uint64_t)(i0 + i), (uint32_t)g, kOmegaTabBf16, b);
      for (int j = 0; j < 8; ++j) z[j] = __uint_as_float((uint32_t)b[j] << 16);
    } else {
      uint32_t c[8];
      omega8_e4m3(seed, (uint64_t)(i0 + i), (uint32_t)g, kOmegaTabE4M3, c);
      for (int j = 0; j < 8; ++j) z[j] = __builtin_amdgcn_cvt_f32_fp8((int)c[j], 0) * (1.0f / 64.0f);
    }
    for (int j = 0; j < 8; ++j)
      if (8 * g + j < ell) reinterpret_cast<float*>(out)[i * ld + 8 * g + j] = z[j];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
constexpr int kNcbF32 = 2;

void sketch_tile_geometry(int prec, int ell, int wide, int* ell_pad, int* n_mt, int* rbw) {
  if (prec == RID_SKETCH_BF16 && wide) {
    // two workgroups per 512-column tile, 32 rbw rows each
    const int rows = (ell + 63) / 64 * 64;
    *n_mt = 2;
    *rbw = rows / 64;
    *ell_pad = rows;
  } else if (prec == RID_SKETCH_BF16 || prec == RID_SKETCH_FP8) {
    // all test-matrix rows in one workgroup up to 320 rows, else split
    const int rows = (ell + 63) / 64 * 64;
    *n_mt = (rows + 319) / 320;
    *rbw = (rows + 64 * *n_mt - 1) / (64 * *n_mt);
    *ell_pad = *n_mt * 64 * *rbw;
  } else {
    *ell_pad = (ell + kMTile - 1) / kMTile * kMTile;
    *n_mt = *ell_pad / kMTile;
    *rbw = 0;
  }
}

int64_t sketch_slab_cap(int prec) {
  return (prec == RID_SKETCH_BF16 || prec == RID_SKETCH_FP8) ? 65536 : (prec == RID_SKETCH_F32 ? 32768 : 16384);
}

int sketch_cols_per_wg(int prec, int wide) {
  if (prec == RID_SKETCH_BF16 && wide) return kWideCols;
  if (prec == RID_SKETCH_BF16 || prec == RID_SKETCH_FP8) return kBf16Cols;
  if (prec == RID_SKETCH_F32) return 4 * kNcbF32 * 32;
  return 64;
}

hipError_t launch_sketch(int prec, const SketchArgs& a, hipStream_t s) {
  const int n_items = a.n_slabs * a.n_mt * a.n_nt;
  const int grid = 8 * ((n_items + 7) / 8);
  if (prec == RID_SKETCH_BF16 && a.wide) {
    switch (a.rbw) {
      case 3: hipLaunchKernelGGL(sketch_bf16w_kernel<3>, dim3(grid), dim3(512), 0, s, a); break;
      case 4: hipLaunchKernelGGL(sketch_bf16w_kernel<4>, dim3(grid), dim3(512), 0, s, a); break;
      case 5: hipLaunchKernelGGL(sketch_bf16w_kernel<5>, dim3(grid), dim3(512), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  else if (prec == RID_SKETCH_BF16) {
    switch (a.rbw) {
      case 1: hipLaunchKernelGGL(sketch_bf16_kernel<1>, dim3(grid), dim3(512), 0, s, a); break;
      case 2: hipLaunchKernelGGL(sketch_bf16_kernel<2>, dim3(grid), dim3(512), 0, s, a); break;
      case 3: hipLaunchKernelGGL(sketch_bf16_kernel<3>, dim3(grid), dim3(512), 0, s, a); break;
      case 4: hipLaunchKernelGGL(sketch_bf16_kernel<4>, dim3(grid), dim3(512), 0, s, a); break;
      case 5: hipLaunchKernelGGL(sketch_bf16_kernel<5>, dim3(grid), dim3(512), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  else if (prec == RID_SKETCH_FP8) {
    switch (a.rbw) {
      case 1: hipLaunchKernelGGL(sketch_fp8_kernel<1>, dim3(grid), dim3(512), 0, s, a); break;
      case 2: hipLaunchKernelGGL(sketch_fp8_kernel<2>, dim3(grid), dim3(512), 0, s, a); break;
      case 3: hipLaunchKernelGGL(sketch_fp8_kernel<3>, dim3(grid), dim3(512), 0, s, a); break;
      case 4: hipLaunchKernelGGL(sketch_fp8_kernel<4>, dim3(grid), dim3(512), 0, s, a); break;
      case 5: hipLaunchKernelGGL(sketch_fp8_kernel<5>, dim3(grid), dim3(512), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  else if (prec == RID_SKETCH_F32)
    hipLaunchKernelGGL(sketch_f32_kernel<kNcbF32>, dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(sketch_f64_kernel, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sketch_reduce(int prec, const SketchArgs& a, hipStream_t s) {
  dim3 grid((a.ell + 63) / 64, a.b);
  if (prec == RID_SKETCH_F64)
    hipLaunchKernelGGL(sketch_reduce_kernel<double>, grid, dim3(64 * kReduceWaves), 0, s, a);
  else
    hipLaunchKernelGGL(sketch_reduce_kernel<float>, grid, dim3(64 * kReduceWaves), 0, s, a);
  return hipGetLastError();
}

namespace {
const void* multi_func(int prec, int rbw, int wide) {
  if (prec == RID_SKETCH_BF16 && wide) {
    switch (rbw) {
      case 3: return reinterpret_cast<const void*>(sketch_bf16w_multi<3>);
      case 4: return reinterpret_cast<const void*>(sketch_bf16w_multi<4>);
      case 5: return reinterpret_cast<const void*>(sketch_bf16w_multi<5>);
      default: return nullptr;
    }
  }
  if (prec == RID_SKETCH_BF16) {
    switch (rbw) {
      case 1: return reinterpret_cast<const void*>(sketch_bf16_multi<1>);
      case 2: return reinterpret_cast<const void*>(sketch_bf16_multi<2>);
      case 3: return reinterpret_cast<const void*>(sketch_bf16_multi<3>);
      case 4: return reinterpret_cast<const void*>(sketch_bf16_multi<4>);
      case 5: return reinterpret_cast<const void*>(sketch_bf16_multi<5>);
      default: return nullptr;
    }
  }
  if (prec == RID_SKETCH_FP8) {
    switch (rbw) {
      case 1: return reinterpret_cast<const void*>(sketch_fp8_multi<1>);
      case 2: return reinterpret_cast<const void*>(sketch_fp8_multi<2>);
      case 3: return reinterpret_cast<const void*>(sketch_fp8_multi<3>);
      case 4: return reinterpret_cast<const void*>(sketch_fp8_multi<4>);
      case 5: return reinterpret_cast<const void*>(sketch_fp8_multi<5>);
      default: return nullptr;
    }
  }
  if (prec == RID_SKETCH_F32) return reinterpret_cast<const void*>(sketch_f32_multi<kNcbF32>);
  return reinterpret_cast<const void*>(sketch_f64_multi);
}
}  // namespace

// One persistent launch per kernel instance (form, rows per workgroup): its
// workgroups walk the work items of every stream of the group.
void plan_sketch_multi(int prec, const SketchArgs* h, int ns, int grid_cap, Stage& st, std::vector<BLaunch>& out) {
  std::vector<char> done(ns, 0);
  for (int i = 0; i < ns; ++i) {
    if (done[i]) continue;
    const void* f = multi_func(prec, h[i].rbw, h[i].wide);
    std::vector<SketchArgs> g;
    std::vector<int> start{0};
    for (int j = i; j < ns; ++j)
      if (!done[j] && multi_func(prec, h[j].rbw, h[j].wide) == f) {
        done[j] = 1;
        g.push_back(h[j]);
        start.push_back(start.back() + h[j].n_slabs * h[j].n_mt * h[j].n_nt);
      }
    if (start.back() == 0) continue;
    BLaunch L{};
    L.func = f;
    L.multi = true;
    L.ns = (int)g.size();
    L.total = start.back();
    L.grid = dim3((unsigned)std::min(L.total, grid_cap));
    L.block = dim3((prec == RID_SKETCH_BF16 || prec == RID_SKETCH_FP8) ? 512 : 256);
    L.lds = 0;
    L.extra = -1;
    L.args = st.put(g.data(), g.size());
    L.aux = st.put(start.data(), start.size());
    L.kind = 0;
    L.bytes = 0.0;
    for (const SketchArgs& a : g) L.bytes += (double)a.b * (double)a.m * (prec == RID_SKETCH_F64 ? 8.0 : 4.0);
    out.push_back(L);
  }
}

void plan_sketch_reduce_b(int prec, const SketchArgs* h, int ns, Stage& st, std::vector<BLaunch>& out) {
  std::vector<SketchArgs> g(h, h + ns);
  std::vector<int4> dims;
  int maxb = 0;
  for (int i = 0; i < ns; ++i) {
    dims.push_back(make_int4((h[i].ell + 63) / 64, h[i].b, 1, 0));
    maxb = std::max(maxb, dims.back().x * dims.back().y);
  }
  if (maxb == 0) return;
  BLaunch L{};
  L.func = prec == RID_SKETCH_F64 ? reinterpret_cast<const void*>(sketch_reduce_kernel_b<double>)
                                  : reinterpret_cast<const void*>(sketch_reduce_kernel_b<float>);
  L.grid = dim3((unsigned)maxb, (unsigned)ns);
  L.block = dim3(64 * kReduceWavesBatch);
  L.extra = -1;
  L.args = st.put(g.data(), g.size());
  L.aux = st.put(dims.data(), dims.size());
  L.kind = 1;
  out.push_back(L);
}

hipError_t launch_omega_block(int prec, uint64_t seed, int ell, int64_t i0, int64_t count,
                              void* out, int64_t ld, hipStream_t s) {
  dim3 grid((unsigned)((count + 255) / 256), (ell + 7) / 8);
  hipLaunchKernelGGL(omega_block_kernel, grid, dim3(256), 0, s, prec, seed, ell, i0, count, out, ld);
  return hipGetLastError();
}

}  // namespace rid
