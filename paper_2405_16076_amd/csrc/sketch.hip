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

namespace rid {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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
// owns row group w&1 (RBW blocks of 32 rows) and the column pair w>>1 (two
// blocks of 32 columns): 2*RBW accumulator tiles.  Per 32-row chunk:
//   * the snapshot chunk (32 rows x 256 columns) is read in 128-byte runs
//     (8 lanes per column), rounded to bfloat16 and stored in LDS;
//   * the matching 64*RBW x 32 tile of Omega is generated (one Philox call per
//     8 rows x 1 data row) into LDS;
// both double-buffered, so chunk c+1 is loaded and generated while the
// matrix cores work on chunk c.
// ---------------------------------------------------------------------------
constexpr int kBf16Cols = 256;

template <int RBW>
__global__ __launch_bounds__(512, 1) void sketch_bf16_kernel(SketchArgs a) {
  constexpr int KC = 32;                 // rows per chunk
  constexpr int MROWS = 64 * RBW;        // test-matrix rows per workgroup
  constexpr int LDA = KC + 8;            // bf16 per LDS row (80 bytes)
  constexpr int NGEN = (MROWS / 8) * KC; // Philox calls per chunk
  __shared__ __attribute__((aligned(16))) uint16_t om[2][MROWS * LDA];
  __shared__ __attribute__((aligned(16))) uint16_t dt[2][kBf16Cols * LDA];
  int slab, mt, nt;
  if (!sketch_item(a, blockIdx.x, slab, mt, nt)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int rg = wave & 1, cp = wave >> 1;
  const int64_t r0 = (int64_t)slab * a.slab_rows;
  const int64_t r1 = min(a.m, r0 + a.slab_rows);
  const int row_base = mt * MROWS;       // first test-matrix row of this workgroup

  // staging: thread -> columns (tid>>3) + 64 i, rows 4 (tid&7) .. +4 of the chunk
  const int scol = tid >> 3, srow = 4 * (tid & 7);
  const gmem_t<float>* sp[4];
  bool sok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = nt * kBf16Cols + scol + 64 * i;
    sok[i] = c < a.b;
    sp[i] = gload_ptr(sok[i] ? reinterpret_cast<const float*>(a.colptr[a.c0 + c]) : nullptr);
  }
  double nrm[4] = {0.0, 0.0, 0.0, 0.0};

  auto load_chunk = [&](int64_t k0, float4 xr[4]) {
    const int64_t row = k0 + srow;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (sok[i] && row + 4 <= r1) {
        xr[i] = gload_f4(sp[i] + row);
      } else {
        xr[i].x = (sok[i] && row + 0 < r1) ? sp[i][row + 0] : 0.0f;
        xr[i].y = (sok[i] && row + 1 < r1) ? sp[i][row + 1] : 0.0f;
        xr[i].z = (sok[i] && row + 2 < r1) ? sp[i][row + 2] : 0.0f;
        xr[i].w = (sok[i] && row + 3 < r1) ? sp[i][row + 3] : 0.0f;
      }
    }
  };
  auto store_chunk = [&](const float4 xr[4], uint16_t* d) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      nrm[i] = fma((double)xr[i].x, (double)xr[i].x, nrm[i]);
      nrm[i] = fma((double)xr[i].y, (double)xr[i].y, nrm[i]);
      nrm[i] = fma((double)xr[i].z, (double)xr[i].z, nrm[i]);
      nrm[i] = fma((double)xr[i].w, (double)xr[i].w, nrm[i]);
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      bf16x4 v = {(__bf16)xr[i].x, (__bf16)xr[i].y, (__bf16)xr[i].z, (__bf16)xr[i].w};
      *reinterpret_cast<bf16x4*>(&d[(scol + 64 * i) * LDA + srow]) = v;
    }
  };
  auto gen = [&](int64_t k0, uint16_t* d) {
    for (int it = tid; it < NGEN; it += 512) {
      const int g = it / KC, k = it % KC;
      uint16_t* dst = d + (8 * g) * LDA + k;
      if (row_base + 8 * g < a.ell) {
        float z[8];
        omega8_f32(a.seed, (uint64_t)(k0 + k), (uint32_t)(row_base / 8 + g), z);
#pragma unroll
        for (int j = 0; j < 8; ++j) dst[j * LDA] = __builtin_bit_cast(uint16_t, (__bf16)z[j]);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) dst[j * LDA] = 0;
      }
    }
  };

  f32x16 acc[RBW][2];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.0f;

  {
    float4 x0[4];
    load_chunk(r0, x0);
    store_chunk(x0, dt[0]);
    gen(r0, om[0]);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = r0; k0 < r1; k0 += KC) {
    const bool more = k0 + KC < r1;
    float4 xn[4];
    if (more) {
      load_chunk(k0 + KC, xn);
      gen(k0 + KC, om[cur ^ 1]);
    }
    const uint16_t* O = om[cur];
    const uint16_t* D = dt[cur];
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      bf16x8 bop[2];
#pragma unroll
      for (int c = 0; c < 2; ++c)
        bop[c] = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const u16x8*>(&D[((2 * cp + c) * 32 + l32) * LDA + 16 * s + 8 * half]));
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
        const bf16x8 av = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const u16x8*>(&O[((rg * RBW + r) * 32 + l32) * LDA + 16 * s + 8 * half]));
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bop[c], acc[r][c], 0, 0, 0);
      }
    }
    if (more) store_chunk(xn, dt[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
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
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double t = nrm[i];
      t += __shfl_xor(t, 1);
      t += __shfl_xor(t, 2);
      t += __shfl_xor(t, 4);
      if (sok[i] && (tid & 7) == 0)
        a.normpart[(int64_t)slab * a.b_max + nt * kBf16Cols + scol + 64 * i] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// binary32 form: v_mfma_f32_32x32x2_f32 (A lane l: row l%32, k = l/32; B lane
// l: column l%32, k = l/32).  Within a 16-row chunk lane half h reads rows
// 8h..8h+7 of its column and MFMA step s uses row 8h+s of both operands.
// ---------------------------------------------------------------------------
template <int NCB>
__global__ __launch_bounds__(256) void sketch_f32_kernel(SketchArgs a) {
  constexpr int KC = 16;
  constexpr int LD = KC + 4;  // floats per LDS tile row (80 bytes)
  __shared__ __attribute__((aligned(16))) float om[kMTile * LD];
  int slab, mt, nt;
  if (!sketch_item(a, blockIdx.x, slab, mt, nt)) return;
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
      omega8_f32_accurate(a.seed, (uint64_t)(k0 + gk), (uint32_t)(mt * (kMTile / 8) + gg), z);
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

// ---------------------------------------------------------------------------
// binary64 form: 64 test-matrix rows x 64 columns per workgroup, 16-row
// chunks staged in LDS, 4 x 4 outputs per thread, binary64 FMA.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sketch_f64_kernel(SketchArgs a) {
  constexpr int KC = 16, NTC = 64;
  __shared__ double om[KC][kMTile + 1];
  __shared__ double dt[KC][NTC + 1];
  int slab, mt, nt;
  if (!sketch_item(a, blockIdx.x, slab, mt, nt)) return;
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

// Fixed-order binary64 sum of the slab partials into S(:, c0:c0+b) and
// ||a_j||^2; a non-finite norm (a non-finite snapshot value) sets the flag.
template <typename T>
__global__ void sketch_reduce_kernel(const T* __restrict__ part, const double* __restrict__ normpart,
                                     int n_slabs, int b_max, int ell_pad, int ell, int b, int64_t c0,
                                     double* __restrict__ S, double* __restrict__ colsq,
                                     int32_t* nonfinite) {
  const int c = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b) return;
  if (r < ell) {
    double s = 0.0;
    for (int sl = 0; sl < n_slabs; ++sl) s += (double)part[((int64_t)sl * b_max + c) * ell_pad + r];
    S[(c0 + c) * ell + r] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double q = 0.0;
    for (int sl = 0; sl < n_slabs; ++sl) q += normpart[(int64_t)sl * b_max + c];
    colsq[c0 + c] = q;
    if (!isfinite(q)) *nonfinite = 1;
  }
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
    if (prec == RID_SKETCH_F32)
      omega8_f32_accurate(seed, (uint64_t)(i0 + i), (uint32_t)g, z);
    else
      omega8_f32(seed, (uint64_t)(i0 + i), (uint32_t)g, z);
    for (int j = 0; j < 8; ++j) {
      float v = z[j];
      if (prec == RID_SKETCH_BF16) v = __uint_as_float((uint32_t)bf16_bits_rne(v) << 16);
      if (8 * g + j < ell) reinterpret_cast<float*>(out)[i * ld + 8 * g + j] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
constexpr int kNcbF32 = 2;

int sketch_cols_per_wg(int prec) {
  if (prec == RID_SKETCH_BF16) return kBf16Cols;
  if (prec == RID_SKETCH_F32) return 4 * kNcbF32 * 32;
  return 64;
}

hipError_t launch_sketch(int prec, const SketchArgs& a, hipStream_t s) {
  const int n_items = a.n_slabs * a.n_mt * a.n_nt;
  const int grid = 8 * ((n_items + 7) / 8);
  if (prec == RID_SKETCH_BF16) {
    switch (a.rbw) {
      case 1: hipLaunchKernelGGL(sketch_bf16_kernel<1>, dim3(grid), dim3(512), 0, s, a); break;
      case 2: hipLaunchKernelGGL(sketch_bf16_kernel<2>, dim3(grid), dim3(512), 0, s, a); break;
      case 3: hipLaunchKernelGGL(sketch_bf16_kernel<3>, dim3(grid), dim3(512), 0, s, a); break;
      case 4: hipLaunchKernelGGL(sketch_bf16_kernel<4>, dim3(grid), dim3(512), 0, s, a); break;
      case 5: hipLaunchKernelGGL(sketch_bf16_kernel<5>, dim3(grid), dim3(512), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  else if (prec == RID_SKETCH_F32)
    hipLaunchKernelGGL(sketch_f32_kernel<kNcbF32>, dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(sketch_f64_kernel, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sketch_reduce(int prec, const SketchArgs& a, int ell, double* S, double* colsq,
                                int32_t* nonfinite, hipStream_t s) {
  dim3 grid((ell + 63) / 64, a.b);
  if (prec == RID_SKETCH_F64)
    hipLaunchKernelGGL(sketch_reduce_kernel<double>, grid, dim3(64), 0, s,
                       reinterpret_cast<const double*>(a.part), a.normpart, a.n_slabs, a.b_max,
                       a.ell_pad, ell, a.b, a.c0, S, colsq, nonfinite);
  else
    hipLaunchKernelGGL(sketch_reduce_kernel<float>, grid, dim3(64), 0, s,
                       reinterpret_cast<const float*>(a.part), a.normpart, a.n_slabs, a.b_max,
                       a.ell_pad, ell, a.b, a.c0, S, colsq, nonfinite);
  return hipGetLastError();
}

hipError_t launch_omega_block(int prec, uint64_t seed, int ell, int64_t i0, int64_t count,
                              void* out, int64_t ld, hipStream_t s) {
  dim3 grid((unsigned)((count + 255) / 256), (ell + 7) / 8);
  hipLaunchKernelGGL(omega_block_kernel, grid, dim3(256), 0, s, prec, seed, ell, i0, count, out, ld);
  return hipGetLastError();
}

}  // namespace rid
