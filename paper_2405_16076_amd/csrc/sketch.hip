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
// (v%4) + 4(l/32) + 8(v/4) for v = 0..15.  Within a 32-row chunk, lane half h
// reads rows 16h..16h+15 of its column; MFMA step s in {0,1} uses rows
// 16h+8s..+8 of both operands (the K order is a permutation shared by both).
// ---------------------------------------------------------------------------
template <int NCB>
__global__ __launch_bounds__(256) void sketch_bf16_kernel(SketchArgs a) {
  constexpr int KC = 32;
  constexpr int LD = KC + 8;  // bf16 per LDS tile row (80 bytes)
  __shared__ __attribute__((aligned(16))) uint16_t om[kMTile * LD];
  int slab, mt, nt;
  if (!sketch_item(a, blockIdx.x, slab, mt, nt)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int64_t r0 = (int64_t)slab * a.slab_rows;
  const int64_t r1 = min(a.m, r0 + a.slab_rows);

  const float* colp[NCB];
  bool ok[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int c = nt * (4 * NCB * 32) + wave * (NCB * 32) + cb * 32 + l32;
    ok[cb] = c < a.b;
    colp[cb] = ok[cb] ? reinterpret_cast<const float*>(a.colptr[a.c0 + c]) : nullptr;
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

  const int gk = tid & 31, gg = tid >> 5;  // Omega generation: row k, group g
  for (int64_t k0 = r0; k0 < r1; k0 += KC) {
    {
      float z[8];
      omega8_f32(a.seed, (uint64_t)(k0 + gk), (uint32_t)(mt * (kMTile / 8) + gg), z);
#pragma unroll
      for (int j = 0; j < 8; ++j) om[(8 * gg + j) * LD + gk] = bf16_bits_rne(z[j]);
    }
    __syncthreads();
    u16x8 bop[NCB][2];
    const int64_t rr = k0 + 16 * half;
    const bool full = (k0 + KC <= r1);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      float x[16];
      if (ok[cb] && full) {
        const float4* p = reinterpret_cast<const float4*>(colp[cb] + rr);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 v = p[q];
          x[4 * q] = v.x;
          x[4 * q + 1] = v.y;
          x[4 * q + 2] = v.z;
          x[4 * q + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = (ok[cb] && rr + j < r1) ? colp[cb][rr + j] : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) nrm[cb] = fma((double)x[j], (double)x[j], nrm[cb]);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        bop[cb][0][j] = bf16_bits_rne(x[j]);
        bop[cb][1][j] = bf16_bits_rne(x[8 + j]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const u16x8 av =
            *reinterpret_cast<const u16x8*>(&om[(rb * 32 + l32) * LD + 16 * half + 8 * s]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bop[cb][s]), acc[rb][cb],
              0, 0, 0);
      }
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

  const float* colp[NCB];
  bool ok[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int c = nt * (4 * NCB * 32) + wave * (NCB * 32) + cb * 32 + l32;
    ok[cb] = c < a.b;
    colp[cb] = ok[cb] ? reinterpret_cast<const float*>(a.colptr[a.c0 + c]) : nullptr;
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
        const float4* p = reinterpret_cast<const float4*>(colp[cb] + rr);
        const float4 v0 = p[0], v1 = p[1];
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
  const double* cp = cok ? reinterpret_cast<const double*>(a.colptr[a.c0 + cglob]) : nullptr;
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
constexpr int kNcbBf16 = 2;  // column blocks of 32 per wave
constexpr int kNcbF32 = 2;

int sketch_cols_per_wg(int prec) {
  if (prec == RID_SKETCH_BF16) return 4 * kNcbBf16 * 32;
  if (prec == RID_SKETCH_F32) return 4 * kNcbF32 * 32;
  return 64;
}

hipError_t launch_sketch(int prec, const SketchArgs& a, hipStream_t s) {
  const int n_items = a.n_slabs * a.n_mt * a.n_nt;
  const int grid = 8 * ((n_items + 7) / 8);
  if (prec == RID_SKETCH_BF16)
    hipLaunchKernelGGL(sketch_bf16_kernel<kNcbBf16>, dim3(grid), dim3(256), 0, s, a);
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
