// The per-update phase of Alg. 3 (every t buffered columns), in binary64:
//   sst_update     SS^T += S_u S_u^T, F += sum ||a_j||^2     (Alg. 3 steps 11, 13)
//   tridiag        Householder tridiagonalisation of SS^T, the top min(k, l)
//                  eigenvalues by Sturm bisection -> ||S_k||^2, the ridge lam,
//                  and the LDL^T factors of T + l*lam*I      (eq. sketch_ridge_leverage_score)
//   scores         tau = s^T (SS^T + l*lam I)^{-1} s for the basis slots and the
//                  buffered columns (Alg. 3 function, steps 17-18)
//   select         prune / fill draws (Alg. 3 steps 19-27)
//   gram           new basis columns into the column pool and their Gram entries
//                  G = A_J^T A_J (Alg. 5 step 1, reused by Alg. 8 step 1)
//   alg4_qr/apply  P = (Omega A_J)^+ (Omega A_obs) by Householder QR (Alg. 4)
//   hutch_*        NA-Hutch++ estimate of ||A_obs - A_J P||_F^2 (Alg. 8)
#include <type_traits>
#include "rid_internal.h"

#include <algorithm>

namespace rid {


// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Sum over the 64 lanes of a wave, returned to every lane, without LDS:
// DPP moves within 16-lane rows (quad xor 1, quad xor 2, half-row mirror,
// row mirror), then the four row sums through readlane, added in a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp_mov_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov_f64<0xB1>(v);   // quad_perm(1,0,3,2)
  v += dpp_mov_f64<0x4E>(v);   // quad_perm(2,3,0,1)
  v += dpp_mov_f64<0x141>(v);  // row_half_mirror
  v += dpp_mov_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Sums over the 64 lanes of N <= 4 per-lane values at once, each returned to
// every lane: the values go to this wave's LDS area red (4 x 64 doubles), 16
// lanes per value add four partials, the 16 lanes of a row add by DPP, and
// lane 16u's total is read back as a scalar.  Cheaper than N wave_sum calls;
// the wave reads only what it wrote, in order, so no barrier is needed.
template <int N>
__device__ __forceinline__ void wave_sum4(double (&v)[N], double* red) {
  static_assert(N >= 1 && N <= 4, "four values per call");
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < N; ++u) red[u * 64 + lane] = v[u];
  const int uu = lane >> 4, j = lane & 15;
  double s = 0.0;
  if (uu < N) s = (red[uu * 64 + j] + red[uu * 64 + j + 16]) + (red[uu * 64 + j + 32] + red[uu * 64 + j + 48]);
  s += dpp_mov_f64<0xB1>(s);   // quad_perm(1,0,3,2)
  s += dpp_mov_f64<0x4E>(s);   // quad_perm(2,3,0,1)
  s += dpp_mov_f64<0x141>(s);  // row_half_mirror
  s += dpp_mov_f64<0x140>(s);  // row_mirror
#pragma unroll
  for (int u = 0; u < N; ++u) v[u] = readlane_f64(s, 16 * u);
}

// Block-wide sum; every thread gets the total.  red must hold blockDim/64 doubles.
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < nw; ++i) tot += red[i];  // fixed order
  return tot;
}

// ---------------------------------------------------------------------------
// Dense binary64 products on the matrix cores (v_mfma_f64_16x16x4f64: A lane
// l holds A(l % 16, l / 16), B lane l holds B(l / 16, l % 16), D lane l
// element v is D(l / 16 + 4 v, l % 16)).  One 32 x 32 tile of C per block of
// four waves; wave w takes the k-steps w, w + 4, ... and the four partial
// tiles are summed in LDS in wave order, so the result does not depend on
// scheduling.  la(m, k) and lb(k, n) return 0 outside the operands.
// ---------------------------------------------------------------------------
typedef double f64x4_m __attribute__((ext_vector_type(4)));

template <typename LA, typename LB>
__device__ __forceinline__ void gemm32_f64(int m0, int n0, int K, LA la, LB lb, double (&out)[2][2][4],
                                           double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  f64x4_m acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4_m{0.0, 0.0, 0.0, 0.0};
  const int nks = (K + 3) / 4;
#pragma unroll 4
  for (int ks = wave; ks < nks; ks += 4) {
    const int k = 4 * ks + k4;
    double av[2], bv[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) av[x] = la(m0 + 16 * x + i16, k);
#pragma unroll
    for (int y = 0; y < 2; ++y) bv[y] = lb(k, n0 + 16 * y + i16);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(((wave * 2 + x) * 2 + y) * 4 + v) * 64 + lane] = acc[x][y][v];
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) s += red[(((w * 2 + x) * 2 + y) * 4 + v) * 64 + lane];
        out[x][y][v] = s;
      }
}

// ---------------------------------------------------------------------------
// SS^T and F of every update of a batch: SS^T_u = SS^T_{u-1} + S_u S_u^T, S_u
// the sketches of update u's own columns, in update order, so SS^T_u does not
// depend on how the updates were grouped into batches.  Slot z of W (and of
// sst_keep) receives update u0 + z, sst_out the state after the last update.
// Block x: one 32 x 32 tile of the upper triangle, mirrored (exactly
// symmetric).  Also starts each update's record.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sst_batch_body(const BatchArgs& b, const Blk bk) {
  __shared__ double red[4 * 16 * 64];
  const int n = b.ell;
  const int nt = (n + 31) / 32;
  int ti = 0, rem = bk.x;
  while (ti < nt && rem >= nt - ti) {
    rem -= nt - ti;
    ++ti;
  }
  const int tj = ti + rem;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  // running sum of this lane's elements of the tile (every wave keeps it)
  double run[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 32 * ti + 16 * x + k4 + 4 * v, c = 32 * tj + 16 * y + i16;
        run[x][y][v] = (r < n && c < n) ? b.sst_in[(int64_t)c * n + r] : 0.0;
      }
  auto store = [&](double* dst) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 32 * ti + 16 * x + k4 + 4 * v, c = 32 * tj + 16 * y + i16;
          if (r < n && c < n && r <= c) {
            dst[(int64_t)c * n + r] = run[x][y][v];
            dst[(int64_t)r * n + c] = run[x][y][v];
          }
        }
  };
  for (int z = 0; z < b.nz; ++z) {
    const int64_t ca = b.c0 + (int64_t)z * b.t;
    const int K = (int)(min((int64_t)(z + 1) * b.t, b.total) - (int64_t)z * b.t);
    const double* Sz = b.S + ca * n;
    double out[2][2][4];
    if (z > 0) __syncthreads();  // the previous product's partials in red have been read
    gemm32_f64(32 * ti, 32 * tj, K, [&](int r, int k) { return (r < n && k < K) ? Sz[(int64_t)k * n + r] : 0.0; },
               [&](int k, int c) { return (k < K && c < n) ? Sz[(int64_t)k * n + c] : 0.0; }, out, red);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) run[x][y][v] += out[x][y][v];
    if (wave == 0) {
      store(b.W + (int64_t)z * n * n);
      if (b.sst_keep) store(b.sst_keep + (int64_t)z * n * n);
    }
  }
  if (wave == 0) store(b.sst_out);
  if (bk.x == 0 && threadIdx.x == 0) {
    // F of update u0 - 1 was written by an earlier launch; the columns are
    // added one by one in stream order
    double F = (b.u0 > 0) ? b.Fu[b.u0 - 1] : 0.0;
    for (int z = 0; z < b.nz; ++z) {
      const int64_t ca = b.c0 + (int64_t)z * b.t;
      const int64_t cend = b.c0 + min((int64_t)(z + 1) * b.t, b.total);
      for (int64_t c = ca; c < cend; ++c) F += b.colsq[c];
      const int64_t u = b.u0 + z;
      b.Fu[u] = F;
      b.skipu[u] = (F > 0.0) ? 0 : 1;
      rid_update* rec = b.recs + u;
      rec->update = u;
      rec->n_obs = cend;
      rec->count = cend - ca;
      rec->F = F;
      rec->flags = (F > 0.0) ? 0 : RID_UPD_SKIPPED;
    }
  }
}

__global__ __launch_bounds__(256) void sst_batch_kernel(BatchArgs b) { sst_batch_body(b, own_block()); }

__global__ __launch_bounds__(256) void sst_batch_kernel_b(Batched<BatchArgs> L) {
  const BatchArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) sst_batch_body(*p, bk);
}

// ---------------------------------------------------------------------------
// Tridiagonalisation (one workgroup of 1024 threads per update), then the
// top eigenvalues by multisection (one wave per eigenvalue, all updates at
// once), then the ridge parameter and LDL^T (one thread per update).
// hv layout: [0,l) reflector tau, [l,2l) d, [2l,3l) e, [3l,4l) Dinv, [4l,5l) L,
// [5l,6l) top eigenvalues (descending).
// ---------------------------------------------------------------------------
// Sturm counts at two shifts, the recurrences interleaved: the number of
// negative pivots of the LDL^T factorisation of T - x I for x = x0 and x1.
// The division by the previous pivot is a reciprocal refined by two Newton
// steps (a few units in the last place, which the count's backward stability
// absorbs; pivots are kept at least pivmin in magnitude, so it stays finite).
__device__ __forceinline__ void sturm_count2(const double* d, const double* e2, int n, double x0, double x1,
                                             double pivmin, int& c0, int& c1) {
  double q0 = d[0] - x0, q1 = d[0] - x1;
  if (fabs(q0) < pivmin) q0 = -pivmin;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  int k0 = q0 < 0.0, k1 = q1 < 0.0;
  for (int i = 1; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
    double r0 = __builtin_amdgcn_rcp(q0), r1 = __builtin_amdgcn_rcp(q1);
    r0 = fma(r0, fma(-q0, r0, 1.0), r0);
    r1 = fma(r1, fma(-q1, r1, 1.0), r1);
    r0 = fma(r0, fma(-q0, r0, 1.0), r0);
    r1 = fma(r1, fma(-q1, r1, 1.0), r1);
    q0 = di - x0 - ei * r0;
    q1 = di - x1 - ei * r1;
    if (fabs(q0) < pivmin) q0 = -pivmin;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    k0 += q0 < 0.0;
    k1 += q1 < 0.0;
  }
  c0 = k0;
  c1 = k1;
}

template <int EMT, int NW>
__device__ __forceinline__ void tridiag_body(const BatchArgs& b, const Blk bk) {
  const int z = bk.x;
  const int64_t u = b.u0 + z;
  const int n = b.ell, tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nw = nth >> 6;
  double* W = b.W + (int64_t)z * n * n;   // holds SS^T of update u on entry
  double* hv = b.hv + (int64_t)z * 6 * n;
  double* htau = hv;
  double* d = hv + n;
  double* e = hv + 2 * n;
  if (b.skipu[u]) {
    if (tid == 0) {
      b.recs[u].sk2 = 0.0;
      b.recs[u].lam = 0.0;
    }
    return;
  }
  // tr(SS^T), the sketch's total energy, before the reduction overwrites W
  if (wv == 0) {
    double part = 0.0;
    for (int k = lane; k < n; k += 64) part += W[(int64_t)k * n + k];
    part = wave_sum(part);
    if (lane == 0) b.tru[u] = part;
  }
  __syncthreads();
  // Householder tridiagonalisation on the lower triangle, one pass over the
  // trailing block per step: iteration j applies the rank-2 update of step
  // j - 1 (A -= v w^T + w v^T, pending) while it forms the reflector and the
  // product p = tau A22 v of step j.  Every wave loads column j, applies the
  // pending update to it and forms the reflector itself (the same operations
  // in the same order, so all waves hold the same v); wave 0 stores it.  Each
  // wave then walks its columns c of the trailing block: loads the column,
  // applies the pending update, stores it, and forms the dot of the column
  // with v (p_c) and adds column c times v_c to its partial of p below the
  // diagonal; the partials meet in LDS in wave order.  Vectors in LDS are
  // indexed by absolute row; in registers element q of a lane is row
  // j + 1 + lane + 64 q.  EMT = ceil(l / 64); the columns of a wave go CB at a
  // time, their loads issued together.  The pass is bound by the SIMDs' issue
  // rate, so per column it keeps to the pending update, the store and two
  // FMAs per row: v_c is a broadcast read of the wave's own copy of v in
  // LDS, and the dots of a batch are summed together (16 lanes per column).
  constexpr int CB = EMT <= 3 ? 4 : (EMT <= 5 ? 3 : (EMT <= 6 ? 2 : 1));
  __shared__ double ppart[NW][kMaxEll];
  __shared__ double dred[NW][4][64];   // a batch's per-lane column dots
  __shared__ double pd[kMaxEll];
  __shared__ double vs[2][kMaxEll];   // reflector of step j at [j & 1]
  __shared__ double ps[2][kMaxEll];   // p of step j at [j & 1]
  double Kp = 0.0;   // K of the pending step
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;            // order of the trailing block, rows j+1..n-1
    const int base = j + 1;
    const bool pend = j > 0;
    const double* Vp = vs[(j + 1) & 1];  // pending step j - 1
    const double* Pp = ps[(j + 1) & 1];
    // pending v and w at this lane's rows
    double pv[EMT], pw[EMT];
#pragma unroll
    for (int q = 0; q < EMT; ++q) {
      const int k = lane + 64 * q;
      const double vv = (pend && k < m) ? Vp[base + k] : 0.0;
      const double pp0 = (pend && k < m) ? Pp[base + k] : 0.0;
      pv[q] = vv;
      pw[q] = pp0 - Kp * vv;
    }
    // column j with the pending update: diagonal and x = rows j+1..n-1
    double* colj = W + (int64_t)j * n;
    double vjc = 0.0, wjc = 0.0;
    if (pend) {
      vjc = Vp[j];
      wjc = Pp[j] - Kp * vjc;
    }
    const double dj = fma(-vjc, wjc, fma(-wjc, vjc, colj[j]));
    double xk[EMT];
#pragma unroll
    for (int q = 0; q < EMT; ++q) {
      const int k = lane + 64 * q;
      xk[q] = (k < m) ? fma(-pv[q], wjc, fma(-pw[q], vjc, colj[base + k])) : 0.0;
    }
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < EMT; ++q) {
      const int k = lane + 64 * q;
      if (k >= 1 && k < m) part = fma(xk[q], xk[q], part);
    }
    const double xn2 = wave_sum(part);
    const double alpha = readlane_f64(xk[0], 0);
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    double cv[EMT];
#pragma unroll
    for (int q = 0; q < EMT; ++q) {
      const int k = lane + 64 * q;
      cv[q] = (k == 0) ? 1.0 : ((k < m) ? xk[q] * scal : 0.0);
    }
    double* vcur = vs[j & 1];
    if (wv == 0) {
#pragma unroll
      for (int q = 0; q < EMT; ++q) {
        const int k = lane + 64 * q;
        if (k < m) vcur[base + k] = cv[q];
      }
      if (lane == 0) {
        htau[j] = tau;
        e[j] = beta;
        d[j] = dj;
      }
    }
    // trailing block: pending update, store, p partials with the new v
    double* A22 = W + (int64_t)base * n + base;  // A22(k, c) = A22[c n + k], k >= c
    // this wave's row of partials holds its copy of v until the pass ends, so
    // v_c is one broadcast read
    double* vloc = ppart[wv];
#pragma unroll
    for (int q = 0; q < EMT; ++q) {
      const int k = lane + 64 * q;
      if (k < m) vloc[k] = cv[q];
    }
    double pp[EMT];
#pragma unroll
    for (int q = 0; q < EMT; ++q) pp[q] = 0.0;
    // the wave index as a scalar, so that column addresses stay in SGPRs
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    for (int c0 = wvu; c0 < m; c0 += CB * nw) {
      double a[CB][EMT];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = c0 + u * nw;
        const double* col = A22 + (int64_t)c * n;
#pragma unroll
        for (int q = 0; q < EMT; ++q) {
          const int k = lane + 64 * q;
          a[u][q] = (c < m && k >= c && k < m) ? col[k] : 0.0;
        }
      }
      double dot[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = c0 + u * nw;
        dot[u] = 0.0;
        if (c >= m) continue;
        double* col = A22 + (int64_t)c * n;
        const double vc_p = pend ? Vp[base + c] : 0.0;
        const double wc_p = pend ? Pp[base + c] - Kp * vc_p : 0.0;
        const double vc = vloc[c];
#pragma unroll
        for (int q = 0; q < EMT; ++q) {
          const int k = lane + 64 * q;
          if (k >= c && k < m) {
            const double x = pend ? fma(-pv[q], wc_p, fma(-pw[q], vc_p, a[u][q])) : a[u][q];
            if (pend) col[k] = x;
            dot[u] = fma(x, cv[q], dot[u]);
            if (k > c) pp[q] = fma(x, vc, pp[q]);
          }
        }
      }
      // the batch's dots: 16 lanes per column add four partials each, then
      // the 16 lanes of a row add by DPP
#pragma unroll
      for (int u = 0; u < CB; ++u) dred[wv][u][lane] = dot[u];
      {
        const int uu = lane >> 4, j = lane & 15;
        double s4 = 0.0;
        if (uu < CB) s4 = (dred[wv][uu][j] + dred[wv][uu][j + 16]) + (dred[wv][uu][j + 32] + dred[wv][uu][j + 48]);
        s4 += dpp_mov_f64<0xB1>(s4);   // quad_perm(1,0,3,2)
        s4 += dpp_mov_f64<0x4E>(s4);   // quad_perm(2,3,0,1)
        s4 += dpp_mov_f64<0x141>(s4);  // row_half_mirror
        s4 += dpp_mov_f64<0x140>(s4);  // row_mirror
        const int cu = c0 + uu * nw;
        if (j == 0 && uu < CB && cu < m) pd[cu] = s4;
      }
    }
#pragma unroll
    for (int q = 0; q < EMT; ++q) {
      const int k = lane + 64 * q;
      if (k < m) ppart[wv][k] = pp[q];
    }
    __syncthreads();
    // every wave has read column j: store the reflector below its first row
    if (wv == 0) {
#pragma unroll
      for (int q = 0; q < EMT; ++q) {
        const int k = lane + 64 * q;
        if (k > 0 && k < m) colj[base + k] = cv[q];
      }
    }
    double* pcur = ps[j & 1];
    for (int k = tid; k < m; k += nth) {
      double sacc = pd[k];
      for (int w = 0; w < nw; ++w) sacc += ppart[w][k];
      pcur[base + k] = tau * sacc;
    }
    __syncthreads();
    double pvs = 0.0;
#pragma unroll
    for (int q = 0; q < EMT; ++q) {
      const int k = lane + 64 * q;
      if (k < m) pvs = fma(pcur[base + k], cv[q], pvs);
    }
    Kp = 0.5 * tau * wave_sum(pvs);
  }
  if (tid == 0) {
    // the last 2 x 2 block with the pending update of step n - 3
    if (n >= 2) {
      double a00 = W[(int64_t)(n - 2) * n + n - 2], a10 = W[(int64_t)(n - 2) * n + n - 1];
      double a11 = W[(int64_t)(n - 1) * n + n - 1];
      if (n >= 3) {
        const double* Vp = vs[(n - 3) & 1];
        const double* Pp = ps[(n - 3) & 1];
        const double v0 = Vp[n - 2], v1 = Vp[n - 1];
        const double w0 = Pp[n - 2] - Kp * v0, w1 = Pp[n - 1] - Kp * v1;
        a00 = fma(-v0, w0, fma(-w0, v0, a00));
        a10 = fma(-v1, w0, fma(-w1, v0, a10));
        a11 = fma(-v1, w1, fma(-w1, v1, a11));
      }
      d[n - 2] = a00;
      e[n - 2] = a10;
      htau[n - 2] = 0.0;
      d[n - 1] = a11;
    } else {
      d[n - 1] = W[(int64_t)(n - 1) * n + n - 1];
    }
    e[n - 1] = 0.0;
    htau[n - 1] = 0.0;
  }
}

// Top eigenvalues of T, the tridiagonal form of SS^T, by multisection: a
// group of GL lanes per eigenvalue (64 / GL groups per wave, 4 waves per
// workgroup (update, y), eigenvalue idx = (4 y + w) 64 / GL + group in
// descending order, idx < k).  Lane r of a group counts the eigenvalues below
// points 2r + 1 and 2r + 2 of the 2 GL equispaced interior points that cut
// the group's interval into 2 GL + 1 parts, and the group keeps the part
// holding its target (Sturm counts are monotone in the shift, so the points
// with count <= target are a prefix).  Stops at a width of one ulp of the
// eigenvalue or 2 eps ||T||, the accuracy of the reduction itself.  A single
// stream's few updates take GL = 64 (fewest rounds on otherwise idle compute
// units); a batch's many take GL = 4 (least work on a full device).
constexpr int kEigWaves = 4;
template <int GL>
__device__ __forceinline__ void tridiag_eig_body(const BatchArgs& b, const Blk bk) {
  constexpr int EPW = 64 / GL;           // eigenvalues per wave
  __shared__ double e2s[kMaxEll];
  __shared__ double ds[kMaxEll];
  const int z = bk.x;
  const int64_t u = b.u0 + z;
  const int n = b.ell, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kk = min(b.k, n);
  if (b.skipu[u] || bk.y * kEigWaves * EPW >= kk) return;  // uniform over the workgroup
  double* hv = b.hv + (int64_t)z * 6 * n;
  const double* d = hv + n;
  const double* e = hv + 2 * n;
  for (int i = tid; i < n; i += blockDim.x) {
    ds[i] = d[i];
    e2s[i] = (i + 1 < n) ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  const int gi = lane / GL, r = lane % GL;
  const int idx = (bk.y * kEigWaves + wv) * EPW + gi;
  if ((bk.y * kEigWaves + wv) * EPW >= kk) return;  // uniform over the wave
  // Gershgorin interval and pivot threshold (minima and maxima are exact in
  // any order)
  double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double r = ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < n) ? fabs(e[i]) : 0.0);
    lo = fmin(lo, ds[i] - r);
    hi = fmax(hi, ds[i] + r);
    emax2 = fmax(emax2, e2s[i]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
    emax2 = fmax(emax2, __shfl_xor(emax2, o));
  }
  const double bnd = fmax(fabs(lo), fabs(hi));
  lo -= 4.0 * 2.220446049250313e-16 * bnd + 1e-300;
  hi += 4.0 * 2.220446049250313e-16 * bnd + 1e-300;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  const double atol = 2.0 * 2.220446049250313e-16 * bnd;
  constexpr int G = 2 * GL + 1;
  const uint64_t gmask = GL == 64 ? ~0ull : ((1ull << (GL & 63)) - 1) << (gi * GL);
  const int target = n - 1 - min(idx, kk - 1);  // ascending index of the idx-th largest
  double aa = lo, bb = hi;
  for (int it = 0; it < 200; ++it) {
    if (bb - aa <= fmax(2.220446049250313e-16 * fmax(fabs(aa), fabs(bb)), atol)) break;
    const double hs = (bb - aa) / G;
    if (!(aa + hs > aa) || !(aa + (G - 1) * hs < bb)) break;
    int c0, c1;
    sturm_count2(ds, e2s, n, aa + (2 * r + 1) * hs, aa + (2 * r + 2) * hs, pivmin, c0, c1);
    const uint64_t bal0 = __ballot(c0 <= target), bal1 = __ballot(c1 <= target);
    const int cnt = __popcll(bal0 & gmask) + __popcll(bal1 & gmask);
    const double na = cnt == 0 ? aa : aa + cnt * hs;
    const double nb = cnt == G - 1 ? bb : aa + (cnt + 1) * hs;
    aa = na;
    bb = nb;
  }
  if (r == 0 && idx < kk) hv[5 * n + idx] = 0.5 * (aa + bb);
}

constexpr int kEigLanesStream = 64;
constexpr int kEigLanesBatch = 4;

__global__ __launch_bounds__(64 * kEigWaves) void tridiag_eig_kernel(BatchArgs b) {
  tridiag_eig_body<kEigLanesStream>(b, own_block());
}

__global__ __launch_bounds__(64 * kEigWaves) void tridiag_eig_kernel_b(Batched<BatchArgs> L) {
  const BatchArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) tridiag_eig_body<kEigLanesBatch>(*p, bk);
}

// ||S_k||^2 (the top-k eigenvalues summed in index order), the ridge
// parameter, and T + l lambda' I = L D L^T of each update: one wave stages
// d, e and the eigenvalues in LDS, one thread runs the recurrences.
__device__ __forceinline__ void tridiag_ridge_body(const BatchArgs& b, const Blk bk) {
  __shared__ double sd[kMaxEll], se[kMaxEll], smu[kMaxEll];
  const int z = bk.x;
  const int64_t u = b.u0 + z;
  if (b.skipu[u]) return;
  const int n = b.ell, tid = threadIdx.x;
  const int kk = min(b.k, n);
  double* hv = b.hv + (int64_t)z * 6 * n;
  for (int i = tid; i < n; i += blockDim.x) {
    sd[i] = hv[n + i];
    se[i] = hv[2 * n + i];
    smu[i] = i < kk ? hv[5 * n + i] : 0.0;
  }
  __syncthreads();
  if (tid != 0) return;
  double* Dinv = hv + 3 * n;
  double* L = hv + 4 * n;
  double sk2 = 0.0;
  for (int i = 0; i < kk; ++i) sk2 += smu[i];
  const double F = b.Fu[u];
  // the ridge parameter: the rank-k tail energy over k, the tail taken as
  // the sketch's own tail fraction (tr(SS^T) - ||S_k||^2) / tr(SS^T) of F
  // (eqs. ridge-leverage-score, sketch_ridge_leverage_score,
  // g_ridge_leverage_score), floored at rho F / k
  const double tr = b.tru[u];
  const double tail = tr > 0.0 ? F * (tr - sk2) / tr : 0.0;
  const double lam = fmax(tail / b.k, b.ridge_floor * F / b.k);
  const double shift = n * lam;
  b.recs[u].sk2 = sk2;
  b.recs[u].lam = lam;
  // T + shift I = L D L^T (T symmetric positive definite for shift > 0)
  double Di = sd[0] + shift;
  Dinv[0] = 1.0 / Di;
  for (int i = 0; i + 1 < n; ++i) {
    const double li = se[i] / Di;
    L[i] = li;
    Di = sd[i + 1] + shift - li * se[i];
    Dinv[i + 1] = 1.0 / Di;
  }
  L[n - 1] = 0.0;
}

__global__ __launch_bounds__(64) void tridiag_ridge_kernel(BatchArgs b) { tridiag_ridge_body(b, own_block()); }

__global__ __launch_bounds__(64) void tridiag_ridge_kernel_b(Batched<BatchArgs> L) {
  const BatchArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) tridiag_ridge_body(*p, bk);
}

template <int EMT>
__global__ __launch_bounds__(1024) void tridiag_kernel(BatchArgs b) { tridiag_body<EMT, 16>(b, own_block()); }

// NW waves per workgroup: 16 when the launch's workgroups fit on the compute
// units one each; 8 (two workgroups per compute unit) when they do not.
template <int EMT, int NW>
__global__ __launch_bounds__(64 * NW) void tridiag_kernel_b(Batched<BatchArgs> L) {
  const BatchArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) tridiag_body<EMT, NW>(*p, bk);
}

// ---------------------------------------------------------------------------
// Sketched ridge leverage scores (eq. sketch_ridge_leverage_score; Alg. 3
// steps 17-19) of the t basis slots (items [0, t)) and the buffered columns
// (items [t, t + cnt)): tau = s^T (SS^T + l lambda' I)^{-1} s = sum_i z_i^2 /
// D_i with L z = Q^T s, where Q T Q^T = SS^T is the tridiagonalisation and
// L D L^T = T + l lambda' I.  Y = Q^T [s_item] for every item at once, with
// Q = H_0 ... H_{l-3} the orthogonal factor of the tridiagonalisation formed
// explicitly (scores_q_kernel: column i of Q is H_0 ... H_{i-1} e_i, one wave
// per column), the product on the matrix cores (scores_gemm_kernel), then the
// L D L^T recurrence per item (scores_fin_kernel).
// ---------------------------------------------------------------------------
// EM = ceil(l / 64) elements of a column per lane.
template <int EM>
__device__ __forceinline__ void scores_q_body(const UpdArgs& a, const Blk bk) {
  const int i = bk.x, n = a.ell, lane = threadIdx.x;
  if (a.skipu[a.u] || i >= n) return;
  const double* htau = a.hv;
  double e[EM];
#pragma unroll
  for (int q = 0; q < EM; ++q) e[q] = (lane + 64 * q == i) ? 1.0 : 0.0;
  // reflector j acts on rows j+1..: v = [1, W[j+2.., j]]
  auto fetch = [&](int jr, double (&v)[EM]) {
    const double* vc = a.W + (int64_t)jr * n;
#pragma unroll
    for (int q = 0; q < EM; ++q) {
      const int r = lane + 64 * q;
      v[q] = (r == jr + 1) ? 1.0 : ((r > jr + 1 && r < n) ? vc[r] : 0.0);
    }
  };
  const int jtop = min(i - 1, n - 3);
  double v[EM], vn[EM];
  double tj = 0.0;
  if (jtop >= 0) {
    fetch(jtop, v);
    tj = htau[jtop];
  }
  for (int jr = jtop; jr >= 0; --jr) {
    double tn = 0.0;
    if (jr > 0) {
      fetch(jr - 1, vn);
      tn = htau[jr - 1];
    }
    if (tj != 0.0) {
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < EM; ++q) part = fma(v[q], e[q], part);
      const double g = tj * wave_sum(part);
#pragma unroll
      for (int q = 0; q < EM; ++q) e[q] = fma(-g, v[q], e[q]);
    }
#pragma unroll
    for (int q = 0; q < EM; ++q) v[q] = vn[q];
    tj = tn;
  }
  double* qc = a.Qs + (int64_t)i * n;
#pragma unroll
  for (int q = 0; q < EM; ++q) {
    const int r = lane + 64 * q;
    if (r < n) qc[r] = e[q];
  }
}

// sketch column of score item `item` (-1: empty basis slot)
__device__ __forceinline__ int64_t score_col(const UpdArgs& a, int item) {
  return (item < a.t) ? a.J[item] : a.c0 + (item - a.t);
}

__device__ __forceinline__ void scores_gemm_body(const UpdArgs& a, const Blk bk) {
  __shared__ double red[4 * 16 * 64];
  __shared__ int64_t cols[32];
  const int n = a.ell, items = a.t + a.cnt;
  if (a.skipu[a.u]) return;
  const int nmt = (n + 31) / 32;
  const int m0 = 32 * (bk.x % nmt), n0 = 32 * (bk.x / nmt);
  if (threadIdx.x < 32) cols[threadIdx.x] = (n0 + (int)threadIdx.x < items) ? score_col(a, n0 + threadIdx.x) : -1;
  __syncthreads();
  const double* Q = a.Qs;
  const double* S = a.S;
  double out[2][2][4];
  gemm32_f64(m0, n0, n, [&](int m, int k) { return (m < n && k < n) ? Q[(int64_t)m * n + k] : 0.0; },
             [&](int k, int c) {
               const int64_t col = cols[c - n0];
               return (k < n && col >= 0) ? S[col * n + k] : 0.0;
             },
             out, red);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave == 0) {
    const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = m0 + 16 * x + k4 + 4 * v, c = n0 + 16 * y + i16;
          if (r < n && c < items) a.Ys[(int64_t)c * n + r] = out[x][y][v];
        }
  }
}

__device__ __forceinline__ void scores_fin_body(const UpdArgs& a, const Blk bk) {
  __shared__ double y[kMaxEll];
  const int item = bk.x, lane = threadIdx.x, n = a.ell;
  if (a.skipu[a.u]) return;
  if (score_col(a, item) < 0) {
    if (lane == 0) {
      a.tauC[item] = __longlong_as_double(0x7FF8000000000000LL);
      a.tauC_hist[a.u * a.t + item] = __longlong_as_double(0x7FF8000000000000LL);
    }
    return;
  }
  const double* ys = a.Ys + (int64_t)item * n;
  for (int i = lane; i < n; i += 64) y[i] = ys[i];
  __syncthreads();
  if (lane == 0) {
    const double* Dinv = a.hv + 3 * n;
    const double* L = a.hv + 4 * n;
    double z = y[0];
    double tau = z * z * Dinv[0];
    for (int i = 1; i < n; ++i) {
      z = y[i] - L[i - 1] * z;
      tau = fma(z * z, Dinv[i], tau);
    }
    if (item < a.t) {
      const double tc = fmin(a.tau_old[item], tau);
      a.tauC[item] = tc;
      a.tauC_hist[a.u * a.t + item] = tc;
    } else {
      a.tauD[item - a.t] = tau;
      a.tauD_hist[a.u * a.t + (item - a.t)] = tau;
    }
  }
}

template <int EM>
__global__ __launch_bounds__(64) void scores_q_kernel(UpdArgs a) { scores_q_body<EM>(a, own_block()); }

// Q of every update of a flush in one launch: block (i, z) forms column i of
// the Q of update a.u + z from that update's slices of W, hv and Qs.
template <int EM>
__global__ __launch_bounds__(64) void scores_q_all_kernel(UpdArgs a) {
  const int z = blockIdx.y;
  UpdArgs b = a;
  b.u = a.u + z;
  b.W = a.W + (int64_t)z * a.ell * a.ell;
  b.hv = a.hv + (int64_t)z * 6 * a.ell;
  b.Qs = a.Qs + (int64_t)z * a.ell * a.ell;
  scores_q_body<EM>(b, Blk{(int)blockIdx.x, 0, 0});
}
template <int EM>
__global__ __launch_bounds__(64) void scores_q_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) scores_q_body<EM>(*p, bk);
}

// f(std::integral_constant<int, EM>) with EM = ceil(l / 64), the elements of
// a column of Q per lane
template <typename F>
static void with_em(int ell, F&& f) {
  switch ((ell + 63) / 64) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
  }
}
__global__ __launch_bounds__(256) void scores_gemm_kernel(UpdArgs a) { scores_gemm_body(a, own_block()); }
__global__ __launch_bounds__(256) void scores_gemm_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) scores_gemm_body(*p, bk);
}
__global__ __launch_bounds__(64) void scores_fin_kernel(UpdArgs a) { scores_fin_body(a, own_block()); }
__global__ __launch_bounds__(64) void scores_fin_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) scores_fin_body(*p, bk);
}

// ---------------------------------------------------------------------------
// Prune / fill (Alg. 3).  One wave: the prune draws of all slots at once,
// then the fills in slot order; the fill scan evaluates 64 candidate draws at
// once and takes the first success.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void select_body(const UpdArgs& a, const Blk bk) {
  // the slot state and the buffer's scores are staged in LDS: the fill scan
  // below is serial over the slots and would otherwise wait on global loads
  __shared__ int used[kMaxT];
  __shared__ int64_t sJ[kMaxT];
  __shared__ double stold[kMaxT], stauD[kMaxT];
  __shared__ int lnew_slot[kMaxT], lnew_src[kMaxT], lslot_src[kMaxT];  // the slot lists, built here
  const int lane = threadIdx.x;
  DevScalars* sc = a.sc;
  const int t = a.t;
  const bool skip = a.skipu[a.u] != 0;
  for (int r = lane; r < kMaxT; r += 64) used[r] = 0;
  for (int r = lane; r < a.cnt; r += 64) stauD[r] = a.tauD[r];
  // prune draws: each slot's decision depends on that slot alone
  int n_pruned = 0;
  for (int i = lane; i < t; i += 64) {
    int64_t Ji = a.J[i];
    double told = a.tau_old[i];
    if (!skip && Ji >= 0) {
      const double tc = a.tauC[i];
      const double p = 1.0 - tc / told;
      const double U = decision_uniform(a.select_seed, (uint32_t)a.u, (uint32_t)i, kPruneDraw);
      if (U < p) {
        Ji = -1;
        told = 1.0;
        ++n_pruned;
      } else {
        told = tc;
      }
    }
    sJ[i] = Ji;
    stold[i] = told;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n_pruned += __shfl_xor(n_pruned, off);
  __syncthreads();
  // fills, in slot order: each empty slot takes the first buffered column,
  // not taken by an earlier slot, whose draw falls below its probability
  int n_new = 0;
  if (!skip) {
    for (int i = 0; i < t; ++i) {
      if (sJ[i] >= 0) continue;
      for (int base = 0; base < a.cnt; base += 64) {
        const int r = base + lane;
        bool hit = false;
        if (r < a.cnt && !used[r]) {
          const double q = fmin(1.0, a.fill_mult * stauD[r]);
          hit = decision_uniform(a.select_seed, (uint32_t)a.u, (uint32_t)i, (uint32_t)r) < q;
        }
        const uint64_t ball = __ballot(hit);
        if (ball) {
          const int rs = base + __ffsll((unsigned long long)ball) - 1;
          if (lane == 0) {
            sJ[i] = a.c0 + rs;
            stold[i] = stauD[rs];
            used[rs] = 1;
            lnew_slot[n_new] = i;
            lnew_src[n_new] = rs;
          }
          __syncthreads();
          ++n_new;
          break;
        }
      }
    }
  }
  __syncthreads();
  for (int i = lane; i < t; i += 64) {
    a.J[i] = sJ[i];
    a.tau_old[i] = stold[i];
    a.J_hist[a.u * t + i] = sJ[i];
  }
  // the slot lists in LDS by all lanes (occupied and old slots compacted in
  // slot order through ballots), then written out once
  for (int i = lane; i < t; i += 64) lslot_src[i] = -1;
  __syncthreads();
  for (int q = lane; q < n_new; q += 64) lslot_src[lnew_slot[q]] = lnew_src[q];
  __syncthreads();
  int n_occ = 0, n_old = 0;
  const uint64_t below = (1ull << lane) - 1;
  for (int base = 0; base < t; base += 64) {
    const int i = base + lane;
    const bool occ = i < t && sJ[i] >= 0;
    const bool old = occ && lslot_src[i] < 0;
    const uint64_t bo = __ballot(occ), bd = __ballot(old);
    if (occ) sc->occ_slot[n_occ + __popcll(bo & below)] = i;
    if (old) sc->old_slot[n_old + __popcll(bd & below)] = i;
    n_occ += __popcll(bo);
    n_old += __popcll(bd);
  }
  for (int i = lane; i < t; i += 64) sc->slot_src[i] = lslot_src[i];
  for (int q = lane; q < n_new; q += 64) {
    sc->new_slot[q] = lnew_slot[q];
    sc->new_src[q] = lnew_src[q];
  }
  if (lane == 0) {
    sc->n_new = n_new;
    sc->n_occ = n_occ;
    rid_update* rec = a.recs + a.u;
    rec->n_pruned = n_pruned;
    rec->n_filled = n_new;
    rec->n_occupied = n_occ;
  }
}

__global__ __launch_bounds__(64) void select_kernel(UpdArgs a) { select_body(a, own_block()); }

__global__ __launch_bounds__(64) void select_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) select_body(*p, bk);
}

// ---------------------------------------------------------------------------
// Gram entries of the new basis columns, fused with their copy into the pool.
// One workgroup of 16 waves per (row slab, tile of up to 160 new slots, tile
// of up to 160 occupied slots), so each basis column is read once per slab.
// Occupied slots are taken in the Gram's list order (new slots first).
// Per 32-row chunk the q columns (new slots, read from the buffered snapshot)
// and the j columns (occupied slots: the snapshot for new ones, the pool for
// kept ones) are staged in LDS in 128-byte runs; 16 x 16 blocks of the tile
// are spread over the waves and accumulated with v_mfma_f64_16x16x4_f64
// (A lane l: row l%16, k = l/16; B lane l: column l%16, k = l/16; D lane l,
// element v: column l%16, row l/16 + 4v).  Products of binary32 data are exact
// in binary64 and all sums are binary64.  When every occupied slot is new the
// two lists coincide and only blocks on or above the diagonal are computed.
// Workgroups of j tile 0 also write the new columns into the pool.
// ---------------------------------------------------------------------------
typedef double f64x4_g __attribute__((ext_vector_type(4)));
constexpr int kGramTile = 160;
constexpr int kGramMaxBlocks = 7;   // ceil(10 * 10 / 16)

template <typename T>
__device__ __forceinline__ void gram_body(const UpdArgs& a, const Blk bk) {
  constexpr int KC = (sizeof(T) == 4) ? 32 : 16;  // rows per chunk
  constexpr int LDC = KC + 1;
  __shared__ T sq[kGramTile * LDC];
  __shared__ T sj[kGramTile * LDC];
  __shared__ int blk[kGramMaxBlocks * 16];
  __shared__ int nblk;
  const DevScalars* sc = a.sc;
  const int n_new = sc->n_new, n_occ = sc->n_occ;
  const int qt = bk.y, jt = bk.z, slab = bk.x;
  if (qt * kGramTile >= n_new || jt * kGramTile >= n_occ) return;
  const int nq = min(kGramTile, n_new - qt * kGramTile);
  const int nj = min(kGramTile, n_occ - jt * kGramTile);
  const bool sym = (n_new == n_occ) && (qt == jt);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int64_t r0 = (int64_t)slab * a.gslab_rows;
  const int64_t r1 = min(a.m, r0 + a.gslab_rows);
  const int QB = (nq + 15) / 16, JB = (nj + 15) / 16;
  if (tid == 0) {
    int n = 0;
    for (int bq = 0; bq < QB; ++bq)
      for (int bj = sym ? bq : 0; bj < JB; ++bj) blk[n++] = bq * 16 + bj;
    nblk = n;
  }
  // staging: thread -> one (column, 4-row group) pair per round
  constexpr int RG = KC / 4;                   // 4-row groups per column
  const int ncol_stage = sym ? nq : nq + nj;   // columns staged per chunk
  __syncthreads();
  f64x4_g acc[kGramMaxBlocks];
#pragma unroll
  for (int b = 0; b < kGramMaxBlocks; ++b) acc[b] = f64x4_g{0.0, 0.0, 0.0, 0.0};
  const T* cpool = reinterpret_cast<const T*>(a.cpool);
  for (int64_t k0 = r0; k0 < r1; k0 += KC) {
    for (int it = tid; it < ncol_stage * RG; it += 1024) {
      const int col = it / RG, rgp = it % RG;
      const int64_t row = k0 + 4 * rgp;
      const gmem_t<T>* src;
      gmem_t<T>* cdst = nullptr;
      T* lds;
      if (col < nq) {
        const int q = qt * kGramTile + col;
        src = gload_ptr(reinterpret_cast<const T*>(a.colptr[a.c0 + sc->new_src[q]]));
        if (jt == 0) cdst = gstore_ptr(reinterpret_cast<T*>(a.cpool) + (int64_t)sc->new_slot[q] * a.ldc);
        lds = sq + col * LDC + 4 * rgp;
      } else {
        const int jj = jt * kGramTile + (col - nq);
        const int slot = gram_slot(sc, jj);
        const int s = sc->slot_src[slot];
        src = gload_ptr((s >= 0) ? reinterpret_cast<const T*>(a.colptr[a.c0 + s]) : cpool + (int64_t)slot * a.ldc);
        lds = sj + (col - nq) * LDC + 4 * rgp;
      }
      T v[4];
      if (row + 4 <= r1) {
        // 16-byte aligned: columns start on 64-element boundaries, rows on 4
        if constexpr (sizeof(T) == 4) {
          const float4 x = gload_f4(src + row);
          v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
          if (cdst) gstore_f4(cdst + row, x);
        } else {
          const double2 x0 = gload_d2(src + row);
          const double2 x1 = gload_d2(src + row + 2);
          v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
          if (cdst) {
            gstore_d2(cdst + row, x0);
            gstore_d2(cdst + row + 2, x1);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          v[j] = (row + j < r1) ? src[row + j] : (T)0;
          if (cdst && row + j < r1) cdst[row + j] = v[j];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) lds[j] = v[j];
    }
    __syncthreads();
    const T* SJ = sym ? sq : sj;
    for (int b = 0; b < kGramMaxBlocks; ++b) {
      const int bi = wave + 16 * b;
      if (bi >= nblk) break;
      const int bq = blk[bi] >> 4, bj = blk[bi] & 15;
      const T* pa = sq + (bq * 16 + i16) * LDC + k4;
      const T* pb = SJ + (bj * 16 + i16) * LDC + k4;
#pragma unroll
      for (int s = 0; s < KC / 4; ++s)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)pa[4 * s], (double)pb[4 * s], acc[b], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = a.gpart + (int64_t)slab * a.t * a.t;
  for (int b = 0; b < kGramMaxBlocks; ++b) {
    const int bi = wave + 16 * b;
    if (bi >= nblk) break;
    const int bq = blk[bi] >> 4, bj = blk[bi] & 15;
    const int jl = bj * 16 + i16;
    if (jl >= nj) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ql = bq * 16 + k4 + 4 * v;
      if (ql < nq) {
        out[(int64_t)(qt * kGramTile + ql) * a.t + jt * kGramTile + jl] = acc[b][v];
        if (sym && bj > bq) out[(int64_t)(jt * kGramTile + jl) * a.t + qt * kGramTile + ql] = acc[b][v];
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void gram_kernel(UpdArgs a) { gram_body<T>(a, own_block()); }

template <typename T>
__global__ __launch_bounds__(1024) void gram_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) gram_body<T>(*p, bk);
}

// ---------------------------------------------------------------------------
// Gram entries for binary32 data.  The staged list is the Gram's column list
// (new slots, then the other occupied ones); the products are its first nq
// columns against all of it, and the reduction needs only the entries (q, j)
// with j >= q or j >= nq, the others being mirrors.  One workgroup of 4 waves
// per (row slab, group of output tiles); a wave owns up to 16 blocks of
// v_mfma_f64_16x16x4_f64.  When every slot is new the tiles are 32 x 32 (2 x 2
// blocks, 4 per wave, upper triangle); otherwise 16 x 32 (1 x 2 blocks, 8 per
// wave, so a few new columns pad to 16 rather than 32), skipping the tiles
// that lie wholly below the diagonal of the new-by-new part.  The columns are
// copied HBM -> LDS by LDS-DMA in 32-row chunks, double-buffered, one chunk
// ahead.  MFMA step s of a chunk pairs lane (i16, k4) with row 8 k4 + s of its
// column, so a lane's eight operands of one column are one contiguous 32-byte
// run (two ds_read_b128).
// Products of binary32 data are exact in binary64 and all sums are binary64.
// Workgroups of tile group 0 also copy the new columns into the pool.
// ---------------------------------------------------------------------------
constexpr int kGramKC = 32;
constexpr int kGramWaves = 4;
constexpr int kGramTPW = 4;                        // 32 x 32 tiles per wave
constexpr int kGramGroup = kGramWaves * kGramTPW;  // 32 x 32 tiles per workgroup

__host__ __device__ inline int gram_stage_cols(int t) { return (t + 7) / 8 * 8; }

// Leading 16 x 32 tiles of tile row r (new columns 16 r .. 16 r + 15) that lie
// wholly below the diagonal of the new-by-new part (columns 32 c .. 32 c + 31
// all new and all before 16 r): they hold no entry the reduction reads.
__device__ inline int gram_skip_tiles(int r, int nq) { return min(r / 2, nq / 32); }

// TX: 16-row blocks of new columns per tile (2: square tiles when every slot
// is new, 1: the general case).  The launch's tile groups, sized for 32 x 32
// tiles, also cover the 16 x 32 ones: twice the tiles per group, at most twice
// as many tile rows.
template <int TX>
__device__ __forceinline__ void gram_f32_tiles(const UpdArgs& a, const Blk bk, const int nq, const int nj) {
  constexpr bool sym = TX == 2;
  extern __shared__ __attribute__((aligned(1024))) float gsm[];
  constexpr int TPW = 4 * 2 / TX;        // tiles per wave
  constexpr int GROUP = kGramWaves * TPW;  // tiles per workgroup
  const DevScalars* sc = a.sc;
  const int TQ = (nq + 16 * TX - 1) / (16 * TX), TJ = (nj + 31) / 32;
  int NT = TQ * (TQ + 1) / 2;
  if (!sym) {
    NT = 0;
    for (int r = 0; r < TQ; ++r) NT += TJ - gram_skip_tiles(r, nq);
  }
  const int g0 = bk.y * GROUP;
  if (g0 >= NT) return;
  const int ncap = gram_stage_cols(a.t);
  const int ncol = nj;
  const int nblk = (ncol + 7) / 8;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i16 = lane & 15, k4 = lane >> 4;
  const int slab = bk.x;
  const int64_t r0 = (int64_t)slab * a.gslab_rows;
  const int64_t r1 = min(a.m, r0 + a.gslab_rows);
  const int nch = (int)((r1 - r0 + kGramKC - 1) / kGramKC);
  const bool ragged = (r1 - r0) % kGramKC != 0;
  const int stage_floats = ncap * kGramKC;
  // column sources (device addresses) of the staged list, in LDS after the two stages
  uint64_t* srcs = reinterpret_cast<uint64_t*>(gsm + 2 * stage_floats);
  const float* cpool = reinterpret_cast<const float*>(a.cpool);
  for (int c = tid; c < nblk * 8; c += kGramWaves * 64) {
    const int cc = c < ncol ? c : 0;  // columns past the list copy column 0 (results dropped)
    const int slot = gram_slot(sc, cc);
    const int s = sc->slot_src[slot];  // >= 0 exactly for the new slots
    const float* pc =
        (s >= 0) ? reinterpret_cast<const float*>(a.colptr[a.c0 + s]) : cpool + (int64_t)slot * a.ldc;
    srcs[c] = reinterpret_cast<uint64_t>(pc);
  }
  // pool slots of the new columns
  int* dslot = reinterpret_cast<int*>(srcs + nblk * 8);
  for (int q = tid; q < nq; q += kGramWaves * 64) dslot[q] = sc->new_slot[q];
  __syncthreads();
  // this wave's DMA blocks: wave, wave + 4, ... (8 columns of 128 bytes each)
  const int ninst = nblk > wave ? (nblk - wave + kGramWaves - 1) / kGramWaves : 0;
  auto issue = [&](int c, int st) {
    const int64_t k0 = r0 + (int64_t)c * kGramKC;
    const uint32_t sb = lds_addr(gsm + st * stage_floats);
    for (int i = 0; i < ninst; ++i) {
      const int col = 8 * (wave + kGramWaves * i) + (lane >> 3);
      int64_t row = k0 + 4 * ((lane & 7) ^ col_swz(col));
      if (row >= r1) row = r0;
      const gmem_t<float>* p = gload_ptr(reinterpret_cast<const float*>(srcs[col]));
      lds_dma16(p + row, __builtin_amdgcn_readfirstlane(sb + (uint32_t)(wave + kGramWaves * i) * 1024u));
    }
  };
  auto fixup = [&](int c, int st) {
    const int64_t k0 = r0 + (int64_t)c * kGramKC;
    for (int i = 0; i < ninst; ++i) {
      const int col = 8 * (wave + kGramWaves * i) + (lane >> 3);
      const int64_t row = k0 + 4 * ((lane & 7) ^ col_swz(col));
      float* slot = gsm + st * stage_floats + col * kGramKC + 4 * (lane & 7);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (row + e >= r1) slot[e] = 0.0f;
    }
  };

  // this wave's tiles
  int tq[TPW], tj[TPW];
  int ntw = 0;
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti) {
    const int tile = g0 + wave + kGramWaves * ti;
    tq[ti] = 0;
    tj[ti] = 0;
    if (tile < NT && tile < g0 + GROUP) {
      int r = 0, rem = tile;
      if (sym) {
        while (rem >= TQ - r) {
          rem -= TQ - r;
          ++r;
        }
        tq[ti] = r;
        tj[ti] = r + rem;
      } else {
        while (rem >= TJ - gram_skip_tiles(r, nq)) {
          rem -= TJ - gram_skip_tiles(r, nq);
          ++r;
        }
        tq[ti] = r;
        tj[ti] = gram_skip_tiles(r, nq) + rem;
      }
      ntw = ti + 1;
    }
  }
  f64x4_g acc[TPW][TX][2];
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
    for (int x = 0; x < TX; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[ti][x][y] = f64x4_g{0.0, 0.0, 0.0, 0.0};

  // eight binary32 rows 8 k4 .. 8 k4 + 7 of staged column c
  auto frag = [&](int st, int c, float out[8]) {
    c = min(c, ncap - 1);
    const float* col = gsm + st * stage_floats + c * kGramKC;
    const int key = col_swz(c);
    const float4 x0 = *reinterpret_cast<const float4*>(col + 4 * ((2 * k4) ^ key));
    const float4 x1 = *reinterpret_cast<const float4*>(col + 4 * ((2 * k4 + 1) ^ key));
    out[0] = x0.x; out[1] = x0.y; out[2] = x0.z; out[3] = x0.w;
    out[4] = x1.x; out[5] = x1.y; out[6] = x1.z; out[7] = x1.w;
  };
  const bool copy_pool = bk.y == 0;
  auto pool_copy = [&](int c, int st) {
    const int64_t k0 = r0 + (int64_t)c * kGramKC;
    float* pool = reinterpret_cast<float*>(a.cpool);
    for (int it = tid; it < nq * 8; it += kGramWaves * 64) {
      const int q = it >> 3, p = it & 7;
      const int64_t row = k0 + 4 * (p ^ col_swz(q));
      const float4 x = *reinterpret_cast<const float4*>(gsm + st * stage_floats + q * kGramKC + 4 * p);
      gmem_t<float>* dst = gstore_ptr(pool + (int64_t)dslot[q] * a.ldc + row);
      if (row + 4 <= r1) {
        gstore_f4(dst, x);
      } else {
        const float xv[4] = {x.x, x.y, x.z, x.w};
        for (int e = 0; e < 4; ++e)
          if (row + e < r1) dst[e] = xv[e];
      }
    }
  };

  issue(0, 0);
  wait_dma_all();
  if (nch == 1 && ragged) fixup(0, 0);
  lds_barrier();
  for (int c = 0; c < nch; ++c) {
    const int cur = c & 1;
    if (c + 1 < nch) issue(c + 1, cur ^ 1);
    // the pool stores go out before the products, so that the wait for the
    // next chunk at the end of the step (vmcnt also counts stores) finds them done
    if (copy_pool) pool_copy(c, cur);
    const int st = cur;
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti) {
      if (ti < ntw) {
        float fa[TX][8], fb[2][8];
#pragma unroll
        for (int x = 0; x < TX; ++x) frag(st, 16 * TX * tq[ti] + 16 * x + i16, fa[x]);
#pragma unroll
        for (int y = 0; y < 2; ++y) frag(st, 32 * tj[ti] + 16 * y + i16, fb[y]);
        // on a diagonal 32 x 32 tile the lower-left block is not needed
        const bool diag = sym && tq[ti] == tj[ti];
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8)
#pragma unroll
          for (int x = 0; x < TX; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              if (!(diag && x == 1 && y == 0))
                acc[ti][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)fa[x][s8], (double)fb[y][s8],
                                                                     acc[ti][x][y], 0, 0, 0);
      }
    }
    wait_dma_all();
    if (ragged && c + 1 == nch - 1) fixup(c + 1, cur ^ 1);
    lds_barrier();
  }

  double* out = a.gpart + (int64_t)slab * a.t * a.t;
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti) {
    if (ti >= ntw) continue;
#pragma unroll
    for (int x = 0; x < TX; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        if (sym && tq[ti] == tj[ti] && x == 1 && y == 0) continue;  // not computed
        const int j = 32 * tj[ti] + 16 * y + i16;
        if (j >= nj) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int q = 16 * TX * tq[ti] + 16 * x + k4 + 4 * v;
          if (q < nq) out[(int64_t)q * a.t + j] = acc[ti][x][y][v];
        }
      }
  }
}

__device__ __forceinline__ void gram_f32_body(const UpdArgs& a, const Blk bk) {
  const int nq = a.sc->n_new, nj = a.sc->n_occ;
  if (nq == 0) return;
  if (nq == nj)
    gram_f32_tiles<2>(a, bk, nq, nj);
  else
    gram_f32_tiles<1>(a, bk, nq, nj);
}

__global__ __launch_bounds__(256, 2) void gram_f32_kernel(UpdArgs a) { gram_f32_body(a, own_block()); }

__global__ __launch_bounds__(256, 2) void gram_f32_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) gram_f32_body(*p, bk);
}

constexpr int kGramReduceWaves = 16;   // slab ranges summed in parallel, then in wave order

// Zero the Gram rows/columns of empty slots, then write the new entries
// (fixed-order sum over slabs), symmetrically.
__device__ __forceinline__ void gram_zero_body(const UpdArgs& a, const Blk bk) {
  const int i = bk.x, j = threadIdx.x;
  if (i >= a.t || j >= a.t) return;
  if (a.J[i] < 0 || a.J[j] < 0) a.G[(int64_t)j * a.t + i] = 0.0;
}

__global__ void gram_zero_kernel(UpdArgs a) { gram_zero_body(a, own_block()); }

__global__ void gram_zero_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) gram_zero_body(*p, bk);
}

// One workgroup of 16 waves per (new slot q, 64 list entries): wave w sums the
// w-th sixteenth of the row slabs in order, then the sixteen sums are added in
// order.
__device__ __forceinline__ void gram_reduce_body(const UpdArgs& a, const Blk bk) {
  __shared__ double part[kGramReduceWaves][64];
  const DevScalars* sc = a.sc;
  const int q = bk.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int jj = bk.y * 64 + lane;
  const int nq = sc->n_new;
  if (q >= nq) return;  // the same for the whole workgroup
  // jj indexes the Gram's list (new slots first); an entry between two new
  // slots is taken from the pair with jj >= q
  const bool act = jj < sc->n_occ && !(jj < nq && jj < q);
  double s = 0.0;
  if (act) {
    const int per = (a.gslabs + kGramReduceWaves - 1) / kGramReduceWaves;
    const int s1 = min(a.gslabs, (w + 1) * per);
#pragma unroll 8
    for (int sl = w * per; sl < s1; ++sl) s += a.gpart[((int64_t)sl * a.gld + q) * a.gld + jj];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w != 0 || !act) return;
  double tot = part[0][lane];
#pragma unroll
  for (int i = 1; i < kGramReduceWaves; ++i) tot += part[i][lane];
  const int si = sc->new_slot[q], sj = gram_slot(sc, jj);
  a.G[(int64_t)sj * a.t + si] = tot;
  a.G[(int64_t)si * a.t + sj] = tot;
}

__global__ void gram_reduce_kernel(UpdArgs a) { gram_reduce_body(a, own_block()); }

__global__ void gram_reduce_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) gram_reduce_body(*p, bk);
}

// ---------------------------------------------------------------------------
// Gram entries of binary32 basis columns on the bfloat16 matrix cores (the
// split form, the default for binary32 data).
//
// Every binary32 value a is split exactly into three bfloat16 pieces:
// a0 = RN(a), a1 = RN(a - a0), a2 = a - a0 - a1.  Both residuals are exact in
// binary32, and a2 has at most 8 significant bits, so a = a0 + a1 + a2 for
// every a of magnitude in [2^-100, 2^60] (and zero).  The product a b is the
// sum of the nine piece products, each exact in binary32 (8-bit significands);
// the three of order >= 3 (a1 b2, a2 b1, a2 b2, together below
// 2^-23 (1 + 2^-7) |a b|) are dropped.  v_mfma_f32_32x32x16_bf16 sums the six
// others over 16 rows.  Per 32-row group the products of order 2, then 1,
// then 0 enter a binary32 accumulator that starts at zero; the two groups of a
// 64-row chunk are added in binary32 and the sum is added to a binary64 sum.
// Counting every binary32 addition as rounded (the worst case of the
// instruction's summation), with u = 2^-24, a group's order-2 and order-1
// products (160 terms of total size below 2^-7 (1 + 2^-6) sum|a b|) add at
// most 1.27 u sum|a b|, its order-0 products (32 additions on partial sums
// below 1.02 sum|a b|) at most 32.7 u sum|a b|, and the addition of the two
// groups at most 1.02 u sum|a b|; so per pair of columns
//   |G_ij - A_i^T A_j| <= (37 u + (m / 64 + slabs) 2^-53) sum_r |a_ri| |a_rj|.
//
// A workgroup of 8 waves owns a row slab (the same slabs as the binary64
// form) and a group of up to 16 of the 32 x 32 tiles (new columns x list
// columns, the tiles wholly below the diagonal of the new-by-new part
// skipped).  Waves 0-3 (one per SIMD) only multiply: each takes the same
// number of tiles (round robin, the last ones repeating tile 0 with their
// results dropped), so no SIMD waits on a larger share.  Waves 4-7 only stage:
// per 64-row chunk each of their threads holds 16 bytes of up to sixteen
// columns (16 lanes per column, so one column's 256 bytes are one coalesced
// run), loaded two chunks ahead into registers; it splits them and writes the
// three bfloat16 planes to LDS (double buffered when they fit), and copies
// the new columns to the pool.  The two roles meet at one barrier per chunk,
// so the splitting of chunk c + 1 runs on the vector ALUs while the matrix
// cores multiply chunk c.  Plane layout: the 64 rows of one column in one
// plane are 128 bytes, eight 16-byte slots of 8 rows, slot s stored at
// s ^ col_swz(c), so the 16-byte operand reads of eight consecutive columns
// hit eight distinct bank groups.  MFMA operand lane l reads rows
// 16 s + 8 (l / 32) .. + 8 of column 32 x + l % 32 (the same rows for A and
// B); D lane l holds column l % 32, rows (v % 4) + 4 (l / 32) + 8 (v / 4).
// ---------------------------------------------------------------------------
constexpr int kGsKC = 64;                      // rows per chunk
constexpr int kGsWaves = 8;                    // 4 multiplying + 4 staging
constexpr int kGsMfmaWaves = 4;
constexpr int kGsMaxTPW = 4;                   // 32 x 32 tiles per multiplying wave
constexpr int kGsGroup = kGsMfmaWaves * kGsMaxTPW;  // tiles per workgroup
static_assert(kGsGroup == kGramRunTiles, "a run's list must fit one workgroup's tiles");
constexpr int kGsPlaneColBytes = kGsKC * 2;    // one column of one plane

typedef __bf16 bf16x8_g __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_g __attribute__((ext_vector_type(2)));
typedef float f32x2_g __attribute__((ext_vector_type(2)));
typedef uint16_t u16x8_g __attribute__((ext_vector_type(8)));
typedef float f32x16_g __attribute__((ext_vector_type(16)));

// Staged columns: 160 (t <= 160, two plane buffers), 192 (two) or 256 (one).
__host__ __device__ inline int gsplit_cols(int t) { return t <= 160 ? 160 : t <= 192 ? 192 : 256; }
__host__ __device__ inline int gsplit_bufs(int t) { return t <= 192 ? 2 : 1; }
__host__ __device__ inline int gsplit_skip(int r, int nq) { return min(r, nq / 32); }

// Tiles of a list of nj columns whose first nq are new.
__host__ __device__ inline int gsplit_tiles(int nq, int nj) {
  const int TQ = (nq + 31) / 32, TJ = (nj + 31) / 32;
  int n = 0;
  for (int r = 0; r < TQ; ++r) n += TJ - gsplit_skip(r, nq);
  return n;
}

size_t gram_split_lds(int t) { return (size_t)gsplit_bufs(t) * 3 * gsplit_cols(t) * kGsPlaneColBytes; }

// Tile groups that cover every call with at most t list columns.
int gram_split_groups(int t) {
  int mx = 0;
  for (int nq = 1; nq <= t; ++nq) mx = std::max(mx, gsplit_tiles(nq, t));
  return (mx + kGsGroup - 1) / kGsGroup;
}

// Two binary32 values -> packed bfloat16 pair (RN) and the two residuals.
__device__ __forceinline__ uint32_t gsplit_pair(float& x, float& y) {
  const bf16x2_g h = __builtin_convertvector(f32x2_g{x, y}, bf16x2_g);
  const uint32_t b = __builtin_bit_cast(uint32_t, h);
  x -= __uint_as_float(b << 16);         // exact
  y -= __uint_as_float(b & 0xFFFF0000u);  // exact
  return b;
}

// The multiplying role: TPW tiles per wave, one barrier per chunk (two when
// the planes are single buffered: the staging waves write between them).
template <int NBUF, int NCOL, int TPW>
__device__ __forceinline__ void gram_split_mfma(const UpdArgs& a, const int slab, const int g0, const int NT,
                                                const int nq, const int nj, const int nch, char* const lds) {
  constexpr int plane_bytes = NCOL * kGsPlaneColBytes;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l32 = lane & 31, hf = lane >> 5;
  const int TJ = (nj + 31) / 32;
  int tq[TPW], tj[TPW];
  bool real[TPW];
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti) {
    const int tile = g0 + wave + kGsMfmaWaves * ti;
    real[ti] = tile < NT;
    int r = 0, rem = real[ti] ? tile : 0;
    while (rem >= TJ - gsplit_skip(r, nq)) {
      rem -= TJ - gsplit_skip(r, nq);
      ++r;
    }
    tq[ti] = r;
    tj[ti] = gsplit_skip(r, nq) + rem;
  }
  // LDS byte offsets of this lane's operand columns, slot key applied per step
  int offa[TPW], offb[TPW], keya[TPW], keyb[TPW];
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti) {
    const int ca = 32 * tq[ti] + l32, cb = 32 * tj[ti] + l32;
    offa[ti] = ca * kGsPlaneColBytes;
    offb[ti] = cb * kGsPlaneColBytes;
    keya[ti] = col_swz(ca);
    keyb[ti] = col_swz(cb);
  }
  double gacc[TPW][16];
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
    for (int v = 0; v < 16; ++v) gacc[ti][v] = 0.0;

  // the staging waves' barriers: one after chunk 0 is in buffer 0, then one
  // per chunk (two when single buffered); this role passes the same number
  lds_barrier();
  for (int c = 0; c < nch; ++c) {
    const char* base = lds + (NBUF == 2 ? (c & 1) : 0) * 3 * plane_bytes;
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti) {
      f32x16_g acc[2];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        bf16x8_g fa[2][3], fb[2][3];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int slot = 2 * (2 * g + s) + hf;
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            fa[s][p] = __builtin_bit_cast(bf16x8_g, *reinterpret_cast<const u16x8_g*>(
                                                       base + p * plane_bytes + offa[ti] + ((slot ^ keya[ti]) << 4)));
            fb[s][p] = __builtin_bit_cast(bf16x8_g, *reinterpret_cast<const u16x8_g*>(
                                                       base + p * plane_bytes + offb[ti] + ((slot ^ keyb[ti]) << 4)));
          }
        }
        f32x16_g x = {};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          x = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s][0], fb[s][2], x, 0, 0, 0);
          x = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s][1], fb[s][1], x, 0, 0, 0);
          x = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s][2], fb[s][0], x, 0, 0, 0);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          x = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s][0], fb[s][1], x, 0, 0, 0);
          x = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s][1], fb[s][0], x, 0, 0, 0);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) x = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s][0], fb[s][0], x, 0, 0, 0);
        acc[g] = x;
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) gacc[ti][v] += (double)(acc[0][v] + acc[1][v]);
    }
    if (NBUF == 1) lds_barrier();
    lds_barrier();
  }

  double* out = a.gpart + (int64_t)slab * a.gld * a.gld;
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti) {
    const int j = 32 * tj[ti] + l32;
    if (!real[ti] || j >= nj) continue;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int q = 32 * tq[ti] + (v & 3) + 4 * hf + 8 * (v >> 2);
      if (q < nq) out[(int64_t)q * a.gld + j] = gacc[ti][v];
    }
  }
}

// The staging role: NCOL / 16 loads per thread per chunk, two chunks ahead
// (one for 256 columns, whose two register sets would not fit).
template <int NBUF, int NCOL>
__device__ __forceinline__ void gram_split_stage(const UpdArgs& a, const int64_t r0, const int64_t r1, const int nq,
                                                 const int nj, const int nch, const bool copy_pool, char* const lds) {
  constexpr int NLD = NCOL / 16;
  constexpr int plane_bytes = NCOL * kGsPlaneColBytes;
  const DevScalars* sc = a.sc;
  const int st = threadIdx.x - 64 * kGsMfmaWaves;  // 0 .. 255
  const int part = st & 15;
  // this thread's columns st / 16 + 16 i.  Staged columns past the list read
  // the pool's first column (valid rows, values ignored: a column of the
  // planes only enters the products of its own tile row or column, which
  // are dropped), so that every load is unconditional.  A column is read
  // where it lives: the running update's new slots in the snapshots, the
  // slots filled earlier in this flush there too (slot_ptr), the others in
  // the pool.  At the last update of a flush the columns outside the pool are
  // copied into it (dsl = their slot); earlier updates copy nothing, so a
  // column that enters and leaves the basis within one flush is never copied.
  const float* cpool = reinterpret_cast<const float*>(a.cpool);
  float* pool = reinterpret_cast<float*>(a.cpool);
  const float* src[NLD];
  int dsl[NLD], off[NLD];
  const GramRun* gl = a.grun;
#pragma unroll
  for (int i = 0; i < NLD; ++i) {
    const int c = (st >> 4) + 16 * i;
    src[i] = cpool;
    dsl[i] = -1;
    if (gl) {
      // an explicit list (a run of updates' Grams in one pass): never a flush's last
      if (c < nj) src[i] = reinterpret_cast<const float*>(gl->ptr[c]);
    } else if (c < nj) {
      const int slot = gram_slot(sc, c);
      const int s = sc->slot_src[slot];  // >= 0 exactly for the new slots
      const float* pcol = cpool + (int64_t)slot * a.ldc;
      src[i] = (s >= 0) ? reinterpret_cast<const float*>(a.colptr[a.c0 + s])
                        : reinterpret_cast<const float*>(a.slot_ptr[slot]);
      if (a.flush_last && src[i] != pcol) dsl[i] = slot;
    }
    off[i] = c * kGsPlaneColBytes + (((part >> 1) ^ col_swz(c)) << 4) + ((part & 1) << 3);
  }
  float4 rawA[NLD], rawB[NLD];
  auto load = [&](int c, float4 (&raw)[NLD]) {
    int64_t row = r0 + (int64_t)c * kGsKC + 4 * part;
    if (row >= r1) row = r0;  // past the slab end: a valid row, zeroed at the split
#pragma unroll
    for (int i = 0; i < NLD; ++i) raw[i] = gload_f4(gload_ptr(src[i] + row));
  };
  // zero the rows past the slab end, copy new columns to the pool, split
  // into the planes of buffer buf
  auto store = [&](int c, int buf, const float4 (&raw)[NLD]) {
    const int64_t row = r0 + (int64_t)c * kGsKC + 4 * part;
    const bool full = r0 + (int64_t)(c + 1) * kGsKC <= r1;  // the same for the workgroup
    char* bp = lds + buf * 3 * plane_bytes;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      float x[4] = {raw[i].x, raw[i].y, raw[i].z, raw[i].w};
      if (full) {
        if (copy_pool && dsl[i] >= 0)
          gstore_f4(gstore_ptr(pool + (int64_t)dsl[i] * a.ldc + row), make_float4(x[0], x[1], x[2], x[3]));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (row + e >= r1) x[e] = 0.0f;
        if (copy_pool && dsl[i] >= 0)
          for (int e = 0; e < 4; ++e)
            if (row + e < r1) gstore_ptr(pool + (int64_t)dsl[i] * a.ldc + row)[e] = x[e];
      }
      uint2 p0, p1, p2;
      p0.x = gsplit_pair(x[0], x[1]);
      p0.y = gsplit_pair(x[2], x[3]);
      p1.x = gsplit_pair(x[0], x[1]);
      p1.y = gsplit_pair(x[2], x[3]);
      p2.x = gsplit_pair(x[0], x[1]);
      p2.y = gsplit_pair(x[2], x[3]);
      *reinterpret_cast<uint2*>(bp + off[i]) = p0;
      *reinterpret_cast<uint2*>(bp + plane_bytes + off[i]) = p1;
      *reinterpret_cast<uint2*>(bp + 2 * plane_bytes + off[i]) = p2;
    }
  };
  // lds_barrier, not __syncthreads: the barrier must not wait for the loads
  // of the next chunks, which stay in flight.  Step c (while the multiplying
  // waves take chunk c): split chunk c + 1, whose register set then takes
  // chunk c + 1 + DEPTH.  Every step issues its loads (past the last chunk
  // they read the last chunk again, unused), so that the compiler's wait
  // before a register set's first use counts the other set's loads as issued
  // after it and leaves them in flight.
  constexpr int DEPTH = NCOL <= 192 ? 2 : 1;
  auto step = [&](int c, float4 (&raw)[NLD]) {
    if (NBUF == 1) lds_barrier();
    if (c + 1 < nch) store(c + 1, NBUF == 2 ? ((c + 1) & 1) : 0, raw);
    load(min(c + 1 + DEPTH, nch - 1), raw);
    lds_barrier();
  };
  if (DEPTH == 2) {
    load(0, rawB);
    store(0, 0, rawB);
    load(min(1, nch - 1), rawA);
    load(min(2, nch - 1), rawB);
    lds_barrier();
    int c = 0;
    for (; c + 1 < nch; c += 2) {
      step(c, rawA);
      step(c + 1, rawB);
    }
    if (c < nch) step(c, rawA);
  } else {
    load(0, rawA);
    store(0, 0, rawA);
    load(min(1, nch - 1), rawA);
    lds_barrier();
    for (int c = 0; c < nch; ++c) step(c, rawA);
  }
}

template <int NBUF, int NCOL>
__device__ __forceinline__ void gram_split_tiles(const UpdArgs& a, const Blk bk) {
  extern __shared__ __attribute__((aligned(1024))) float gsm[];
  int nq = a.sc->n_new, nj = a.sc->n_occ;
  if (const GramRun* gl = a.grun) {
    nq = gl->nq;
    nj = gl->nj;
  }
  if (nq == 0) return;
  const int NT = gsplit_tiles(nq, nj);
  const int g0 = bk.y * kGsGroup;
  if (g0 >= NT) return;
  const int slab = bk.x;
  const int64_t r0 = (int64_t)slab * a.gslab_rows;
  const int64_t r1 = min(a.m, r0 + a.gslab_rows);
  const int nch = (int)((r1 - r0 + kGsKC - 1) / kGsKC);
  char* const lds = reinterpret_cast<char*>(gsm);
  if (threadIdx.x < 64 * kGsMfmaWaves) {
    const int tpw = (min(kGsGroup, NT - g0) + kGsMfmaWaves - 1) / kGsMfmaWaves;
    switch (tpw) {
      case 1: gram_split_mfma<NBUF, NCOL, 1>(a, slab, g0, NT, nq, nj, nch, lds); break;
      case 2: gram_split_mfma<NBUF, NCOL, 2>(a, slab, g0, NT, nq, nj, nch, lds); break;
      case 3: gram_split_mfma<NBUF, NCOL, 3>(a, slab, g0, NT, nq, nj, nch, lds); break;
      default: gram_split_mfma<NBUF, NCOL, 4>(a, slab, g0, NT, nq, nj, nch, lds); break;
    }
  } else {
    gram_split_stage<NBUF, NCOL>(a, r0, r1, nq, nj, nch, bk.y == 0, lds);
  }
}

// One kernel per staging shape (t <= 160, t <= 192, larger), so that each
// gets its own register allocation.
template <int NBUF, int NCOL>
__global__ __launch_bounds__(64 * kGsWaves, 1) void gram_split_kernel(UpdArgs a) {
  gram_split_tiles<NBUF, NCOL>(a, own_block());
}

template <int NBUF, int NCOL>
__global__ __launch_bounds__(64 * kGsWaves, 1) void gram_split_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) gram_split_tiles<NBUF, NCOL>(*p, bk);
}

// After the split Gram of an update: the slots it filled point at their
// snapshots in the flush's buffer; after the last update of a flush every
// slot points at its pool column again (the Gram, or gram_pool_flush when the
// update brought no column, has copied them).  One block of kMaxT threads.
__device__ __forceinline__ void gram_ptr_body(const UpdArgs& a, const Blk bk) {
  (void)bk;
  const int i = threadIdx.x;
  if (i >= a.t) return;
  const int s = a.sc->slot_src[i];
  const float* pcol = reinterpret_cast<const float*>(a.cpool) + (int64_t)i * a.ldc;
  if (a.flush_last)
    a.slot_ptr[i] = reinterpret_cast<uint64_t>(pcol);
  else if (s >= 0)
    a.slot_ptr[i] = a.colptr[a.c0 + s];
}

__global__ void gram_ptr_kernel(UpdArgs a) { gram_ptr_body(a, own_block()); }

__global__ void gram_ptr_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) gram_ptr_body(*p, bk);
}

// The last update of a flush that brought no column runs no split Gram: copy
// the occupied slots whose column still lives in the flush's buffer into the
// pool.  Grid (kPoolFlushBlocks, t) of 256 threads, 16 bytes per thread and
// step (columns start on 16-byte boundaries; a ragged last run is copied
// element by element).
constexpr int kPoolFlushBlocks = 64;

__device__ __forceinline__ void gram_pool_flush_body(const UpdArgs& a, const Blk bk) {
  if (!a.flush_last || a.sc->n_new != 0) return;  // the Gram copied them
  const int slot = bk.y;
  if (slot >= a.t || a.J[slot] < 0) return;
  float* pcol = reinterpret_cast<float*>(a.cpool) + (int64_t)slot * a.ldc;
  const float* src = reinterpret_cast<const float*>(a.slot_ptr[slot]);
  if (src == pcol) return;
  const int64_t step = (int64_t)kPoolFlushBlocks * blockDim.x * 4;
  for (int64_t r = ((int64_t)bk.x * blockDim.x + threadIdx.x) * 4; r < a.m; r += step) {
    if (r + 4 <= a.m) {
      gstore_f4(gstore_ptr(pcol + r), gload_f4(gload_ptr(src + r)));
    } else {
      for (int64_t e = r; e < a.m; ++e) pcol[e] = src[e];
    }
  }
}

__global__ __launch_bounds__(256) void gram_pool_flush_kernel(UpdArgs a) { gram_pool_flush_body(a, own_block()); }

__global__ __launch_bounds__(256) void gram_pool_flush_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) gram_pool_flush_body(*p, bk);
}

// ---------------------------------------------------------------------------
// The split Grams of a run of consecutive updates ua .. ub of a flush.  Update
// v's Gram needs the columns new at v against its basis; every such column is
// in [new at ub, ..., new at ua, the others occupied at ua], so when that list
// fits one workgroup's tiles one pass reads it once for the whole run.  In
// that order each entry has the operands it has in the updates' own calls
// (the column that entered later as the tile row; the columns new at one
// update in their order), so its sum is bitwise the same in or out of a run.
// Runs after the selections of the run (no selection reads G).
// ---------------------------------------------------------------------------
// The list of the run of nu updates ending at a.u, from their selection
// states: a column new at v is read from its snapshot (colptr), the others
// where slot_ptr points before the run.  A list column keeps its slot at a
// later update while the slot holds the same column.  One block.
__global__ void gram_run_list_kernel(UpdArgs a, int nu, const DevScalars* sc_hist, const int64_t* J_hist,
                                     GramRun* R) {
  const int64_t ua = a.u - nu + 1;
  __shared__ int q0s[kGramRunMax], q1s[kGramRunMax], nqs;  // list rows new at update ua + w
  if (threadIdx.x == 0) {
    int o = 0;
    for (int w = nu - 1; w >= 0; --w) {
      q0s[w] = o;
      o += sc_hist[ua + w].n_new;
      q1s[w] = o;
      R->q0[w] = q0s[w];
      R->q1[w] = o;
    }
    nqs = o;
    R->nq = o;
    R->nj = o + sc_hist[ua].n_occ - sc_hist[ua].n_new;
    R->nu = nu;
  }
  __syncthreads();
  const int nq = nqs, nj = nq + sc_hist[ua].n_occ - sc_hist[ua].n_new;
  for (int c = threadIdx.x; c < nj; c += blockDim.x) {
    int v = -1, sl;
    uint64_t p;
    if (c < nq) {
      v = 0;
      while (!(c >= q0s[v] && c < q1s[v])) ++v;
      const DevScalars* sv = sc_hist + ua + v;
      const int i = c - R->q0[v];
      sl = sv->new_slot[i];
      p = a.colptr[(ua + v) * a.t + sv->new_src[i]];
    } else {
      v = 0;
      sl = sc_hist[ua].old_slot[c - nq];
      p = a.slot_ptr[sl];
    }
    R->ptr[c] = p;
    const int64_t col = J_hist[(ua + v) * a.t + sl];
    for (int w = 0; w < nu; ++w)
      R->slot[w][c] = (w >= v && J_hist[(ua + w) * a.t + sl] == col) ? sl : -1;
  }
}

// Update entries of G from a run's partials: the list rows new at update w of
// the run against the list columns in its basis.  An entry between two list
// rows lies in the tile of the smaller row; two new columns of this update
// are written once, from the smaller.  Grid (t, list chunks of 64) of 16
// waves, the slab sums as in gram_reduce.
__device__ __forceinline__ void gram_reduce_run_body(const UpdArgs& a, const Blk bk) {
  __shared__ double part[kGramReduceWaves][64];
  const GramRun* R = a.grun;
  const int w = a.grun_u, q0 = R->q0[w], q1 = R->q1[w];
  const int q = q0 + bk.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (q >= q1) return;  // the same for the whole workgroup
  const int jj = bk.y * 64 + lane;
  const bool act = jj < R->nj && R->slot[w][jj] >= 0 && !(jj >= q0 && jj < q1 && jj < q);
  const bool low = jj < R->nq && jj < q;
  const int r = low ? jj : q, c = low ? q : jj;
  double s = 0.0;
  if (act) {
    const int per = (a.gslabs + kGramReduceWaves - 1) / kGramReduceWaves;
    const int s1 = min(a.gslabs, (wv + 1) * per);
#pragma unroll 8
    for (int sl = wv * per; sl < s1; ++sl) s += a.gpart[((int64_t)sl * a.gld + r) * a.gld + c];
  }
  part[wv][lane] = s;
  __syncthreads();
  if (wv != 0 || !act) return;
  double tot = part[0][lane];
#pragma unroll
  for (int i = 1; i < kGramReduceWaves; ++i) tot += part[i][lane];
  const int si = R->slot[w][q], sj = R->slot[w][jj];
  a.G[(int64_t)sj * a.t + si] = tot;
  a.G[(int64_t)si * a.t + sj] = tot;
}

__global__ void gram_reduce_run_kernel(UpdArgs a) { gram_reduce_run_body(a, own_block()); }

static const void* gram_split_fn(int t, bool batched) {
  if (t <= 160)
    return batched ? reinterpret_cast<const void*>(gram_split_kernel_b<2, 160>)
                   : reinterpret_cast<const void*>(gram_split_kernel<2, 160>);
  if (t <= 192)
    return batched ? reinterpret_cast<const void*>(gram_split_kernel_b<2, 192>)
                   : reinterpret_cast<const void*>(gram_split_kernel<2, 192>);
  return batched ? reinterpret_cast<const void*>(gram_split_kernel_b<1, 256>)
                 : reinterpret_cast<const void*>(gram_split_kernel<1, 256>);
}

// ---------------------------------------------------------------------------
// Alg. 4: Householder QR of Omega A_J (occupied slots in slot order), then
// P = R^{-1} Q^T S column by column.  Columns whose pivot |R_ii| falls to
// max(l, n) eps max|R| are dropped from the solve (flag RID_UPD_RANK_DEFICIENT).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void alg4_qr_body(const UpdArgs& a, const Blk bk) {
  __shared__ double red[16];
  __shared__ double v[kMaxEll];
  const int n = a.ell, tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nw = nth >> 6;
  DevScalars* sc = a.sc;
  const int no = sc->n_occ;
  double* A = a.QR;
  for (int64_t idx = tid; idx < (int64_t)n * no; idx += nth) {
    const int jj = (int)(idx / n), r = (int)(idx % n);
    A[(int64_t)jj * n + r] = a.S[a.J[sc->occ_slot[jj]] * n + r];
  }
  __syncthreads();
  for (int jj = 0; jj < no && jj < n; ++jj) {
    double* x = A + (int64_t)jj * n + jj;
    const int len = n - jj;
    double part = 0.0;
    for (int i = 1 + tid; i < len; i += nth) part += x[i] * x[i];
    const double xn2 = block_sum(part, red);
    const double alpha = x[0];
    double tau = 0.0, beta = alpha;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tau = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
      for (int i = tid; i < len; i += nth) v[i] = (i == 0) ? 1.0 : x[i] * scal;
    } else {
      for (int i = tid; i < len; i += nth) v[i] = (i == 0) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int i = 1 + tid; i < len; i += nth) x[i] = v[i];
    if (tid == 0) {
      x[0] = beta;
      a.qr_tau[jj] = tau;
    }
    if (tau != 0.0) {
      for (int c = jj + 1 + wv; c < no; c += nw) {
        double* y = A + (int64_t)c * n + jj;
        double s = 0.0;
        for (int i = lane; i < len; i += 64) s = fma(v[i], y[i], s);
        const double g = tau * wave_sum(s);
        for (int i = lane; i < len; i += 64) y[i] -= g * v[i];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    double rmax = 0.0;
    const int nd = min(no, n);
    for (int i = 0; i < nd; ++i) rmax = fmax(rmax, fabs(A[(int64_t)i * n + i]));
    const double tol = (double)max(n, no) * 2.220446049250313e-16 * rmax;
    int rank = 0;
    for (int i = 0; i < nd; ++i) rank += (fabs(A[(int64_t)i * n + i]) > tol);
    sc->rank = rank;
    if (rank < no) a.recs[a.u].flags |= RID_UPD_RANK_DEFICIENT;
  }
}

__global__ __launch_bounds__(1024) void alg4_qr_kernel(UpdArgs a) { alg4_qr_body(a, own_block()); }

__global__ __launch_bounds__(1024) void alg4_qr_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) alg4_qr_body(*p, bk);
}

// The same factorization with Omega A_J held in registers: column c lives in
// wave c % NW (slot c / NW), row r in lane r % 64 (element r / 64).  Step jj:
// the owner wave of column jj forms the reflector and publishes it in LDS
// (double-buffered by step parity), one barrier, then every wave applies it to
// its own columns still to be reduced (c > jj), over the row chunks that
// reach row jj.  E = ceil(l / 64), NS = ceil(t / NW).

template <int E, int NS, int NW>
__device__ __forceinline__ void alg4_qr_reg_body(const UpdArgs& a, const Blk bk) {
  __shared__ double vb[2][64 * E];
  __shared__ double tb[2];
  __shared__ double qred[NW][4 * 64];   // each wave's dot sums (wave_sum4)
  const int n = a.ell, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  DevScalars* sc = a.sc;
  const int no = sc->n_occ;
  double col[NS][E];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = wave + NW * s;
    const double* src = (c < no) ? a.S + a.J[sc->occ_slot[c]] * n : nullptr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int r = lane + 64 * e;
      col[s][e] = (c < no && r < n) ? src[r] : 0.0;
    }
  }
  const int nsteps = min(no, n);
  for (int jj = 0; jj < nsteps; ++jj) {
    const int ow = jj % NW, os = jj / NW, buf = jj & 1;
    if (wave == ow) {
      double x[E];
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == os)
#pragma unroll
          for (int e = 0; e < E; ++e) x[e] = col[s][e];
      double part = 0.0, al = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = lane + 64 * e;
        if (r > jj && r < n) part = fma(x[e], x[e], part);
        if (e == jj / 64) al = x[e];
      }
      const double xn2 = wave_sum(part);
      const double alpha = __shfl(al, jj & 63);
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xn2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = lane + 64 * e;
        const double vr = (r == jj) ? 1.0 : ((r > jj && r < n) ? x[e] * scal : 0.0);
        vb[buf][r] = vr;
        if (r == jj) x[e] = beta;
        else if (r > jj) x[e] = vr;
      }
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == os)
#pragma unroll
          for (int e = 0; e < E; ++e) col[s][e] = x[e];
      if (lane == 0) {
        tb[buf] = tau;
        a.qr_tau[jj] = tau;
      }
    }
    __syncthreads();
    const double tau = tb[buf];
    if (tau != 0.0) {
      double v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = lane + 64 * e;
        v[e] = (r >= jj && r < n) ? vb[buf][r] : 0.0;
      }
      // Only columns c > jj take the reflector, and v is zero above row jj:
      // batches whose columns are all done and row chunks wholly above jj are
      // skipped by scalar branches (their terms are exact zeros).
      constexpr int B = (E >= 5) ? 4 : 8;
      const int e0 = jj >> 6;
#pragma unroll
      for (int s0 = 0; s0 < NS; s0 += B) {
        if (wave + NW * min(s0 + B - 1, NS - 1) <= jj) continue;
        double d[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
          d[i] = 0.0;
          if (s0 + i < NS)
#pragma unroll
            for (int e = 0; e < E; ++e)
              if (e >= e0) d[i] = fma(v[e], col[s0 + i][e], d[i]);
        }
#pragma unroll
        for (int h = 0; h < B; h += 4) {
          double d4[4] = {d[h], d[h + 1], d[h + 2], d[h + 3]};
          wave_sum4<4>(d4, qred[wave]);
#pragma unroll
          for (int u = 0; u < 4; ++u) d[h + u] = d4[u];
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
          if (s0 + i < NS) {
            const int c = wave + NW * (s0 + i);
            if (c > jj && c < no) {
              const double g = tau * d[i];
#pragma unroll
              for (int e = 0; e < E; ++e)
                if (e >= e0) col[s0 + i][e] = fma(-g, v[e], col[s0 + i][e]);
            }
          }
        }
      }
    }
  }
  double* A = a.QR;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = wave + NW * s;
    if (c < no)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = lane + 64 * e;
        if (r < n) A[(int64_t)c * n + r] = col[s][e];
      }
  }
  __syncthreads();
  if (tid == 0) {
    double rmax = 0.0;
    const int nd = min(no, n);
    for (int i = 0; i < nd; ++i) rmax = fmax(rmax, fabs(A[(int64_t)i * n + i]));
    const double tol = (double)max(n, no) * 2.220446049250313e-16 * rmax;
    int rank = 0;
    for (int i = 0; i < nd; ++i) rank += (fabs(A[(int64_t)i * n + i]) > tol);
    sc->rank = rank;
    if (rank < no) a.recs[a.u].flags |= RID_UPD_RANK_DEFICIENT;
  }
}

template <int E, int NS, int NW>
__global__ __launch_bounds__(64 * NW) void alg4_qr_reg_kernel(UpdArgs a) { alg4_qr_reg_body<E, NS, NW>(a, own_block()); }

template <int E, int NS, int NW>
__global__ __launch_bounds__(64 * NW) void alg4_qr_reg_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) alg4_qr_reg_body<E, NS, NW>(*p, bk);
}

// One wave per observed column c: z = Q^T S(:, c), back substitution, scatter.
__device__ __forceinline__ void alg4_apply_body(const UpdArgs& a, const Blk bk) {
  __shared__ double y[kMaxEll];
  const int64_t c = bk.x;
  const int lane = threadIdx.x, n = a.ell;
  const DevScalars* sc = a.sc;
  const int no = min(sc->n_occ, n);
  double* Pc = a.P + c * a.t;
  for (int i = lane; i < a.t; i += 64) Pc[i] = 0.0;
  if (no == 0) return;
  const double* A = a.QR;
  const double* s = a.S + c * n;
  for (int i = lane; i < n; i += 64) y[i] = s[i];
  __syncthreads();
  for (int jj = 0; jj < no; ++jj) {
    const double tj = a.qr_tau[jj];
    if (tj == 0.0) continue;
    const double* vc = A + (int64_t)jj * n;
    double part = 0.0;
    for (int i = jj + lane; i < n; i += 64) part = fma((i == jj) ? 1.0 : vc[i], y[i], part);
    const double g = tj * wave_sum(part);
    __syncthreads();
    for (int i = jj + lane; i < n; i += 64) y[i] -= g * ((i == jj) ? 1.0 : vc[i]);
    __syncthreads();
  }
  // R x = y(0:no), dropping columns with negligible pivots
  double rmax = 0.0;
  for (int i = 0; i < no; ++i) rmax = fmax(rmax, fabs(A[(int64_t)i * n + i]));
  const double tol = (double)max(n, sc->n_occ) * 2.220446049250313e-16 * rmax;
  for (int i = no - 1; i >= 0; --i) {
    const double rii = A[(int64_t)i * n + i];
    const double xi = (fabs(rii) > tol) ? y[i] / rii : 0.0;
    __syncthreads();
    for (int r = lane; r < i; r += 64) y[r] -= xi * A[(int64_t)i * n + r];
    if (lane == 0) Pc[sc->occ_slot[i]] = xi;
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void alg4_apply_kernel(UpdArgs a) { alg4_apply_body(a, own_block()); }

__global__ __launch_bounds__(64) void alg4_apply_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) alg4_apply_body(*p, bk);
}


// ---------------------------------------------------------------------------
// Alg. 4 as products (t <= kAlg4Gemm): P(occupied, :) = R'^{-1} Q^T S, where
// Q is the thin orthogonal factor of Omega A_J and R' its triangular factor
// without the columns of negligible pivot (their rows of P are zero, as in
// alg4_apply_kernel):
//   alg4_q_kernel    column j of Q = H_0 ... H_j e_j (one wave per column);
//   alg4_m_kernel    M = R'^{-1} Q^T, one wave per row of Q, column-oriented
//                    back substitution against R packed in LDS;
//   alg4_pgemm       P = M S on the matrix cores, scattered to slot order;
//                    rows of empty slots are zeroed.
// ---------------------------------------------------------------------------

// dynamic LDS of alg4_m_kernel: R packed by columns (t of them at most)
inline size_t alg4_m_lds(int t) { return (size_t)t * (t + 1) / 2 * sizeof(double); }

__device__ __forceinline__ void alg4_q_body(const UpdArgs& a, const Blk bk) {
  constexpr int EM = kMaxEll / 64;
  const int j = bk.x, n = a.ell, lane = threadIdx.x;
  const int no = min(a.sc->n_occ, n);
  if (j >= no) return;
  double e[EM];
#pragma unroll
  for (int q = 0; q < EM; ++q) e[q] = (lane + 64 * q == j) ? 1.0 : 0.0;
  // reflector jj - 1 is fetched while reflector jj is applied
  auto fetch = [&](int jj, double (&v)[EM]) {
    const double* vc = a.QR + (int64_t)jj * n;
#pragma unroll
    for (int q = 0; q < EM; ++q) {
      const int r = lane + 64 * q;
      v[q] = (r == jj) ? 1.0 : ((r > jj && r < n) ? vc[r] : 0.0);
    }
  };
  double v[EM], vn[EM];
  fetch(j, v);
  double tj = a.qr_tau[j];
  for (int jj = j; jj >= 0; --jj) {
    double tn = 0.0;
    if (jj > 0) {
      fetch(jj - 1, vn);
      tn = a.qr_tau[jj - 1];
    }
    if (tj != 0.0) {
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < EM; ++q) part = fma(v[q], e[q], part);
      const double g = tj * wave_sum(part);
#pragma unroll
      for (int q = 0; q < EM; ++q) e[q] = fma(-g, v[q], e[q]);
    }
#pragma unroll
    for (int q = 0; q < EM; ++q) v[q] = vn[q];
    tj = tn;
  }
#pragma unroll
  for (int q = 0; q < EM; ++q) {
    const int r = lane + 64 * q;
    if (r < n) a.Qm[(int64_t)j * n + r] = e[q];
  }
}

__device__ __forceinline__ void alg4_m_body(const UpdArgs& a, const Blk bk) {
  constexpr int EY = (kAlg4Gemm + 63) / 64;
  extern __shared__ __attribute__((aligned(16))) double rp[];  // t (t + 1) / 2 doubles
  const int n = a.ell, t = a.t;
  const int no = min(a.sc->n_occ, n);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // R packed by columns: column k at k (k + 1) / 2, rows 0..k
  const int np = no * (no + 1) / 2;
  for (int idx = tid; idx < np; idx += 256) {
    int k = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while (k * (k + 1) / 2 > idx) --k;
    while ((k + 1) * (k + 2) / 2 <= idx) ++k;
    const int i = idx - k * (k + 1) / 2;
    rp[idx] = a.QR[(int64_t)k * n + i];
  }
  __syncthreads();
  double rmax = 0.0;
  for (int i = lane; i < no; i += 64) rmax = fmax(rmax, fabs(rp[i * (i + 1) / 2 + i]));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
  const double tol = (double)max(n, a.sc->n_occ) * 2.220446049250313e-16 * rmax;
  const int r = bk.x * 4 + wave;  // row of Q = column of M
  if (r >= n) return;
  double y[EY];
#pragma unroll
  for (int q = 0; q < EY; ++q) {
    const int i = lane + 64 * q;
    y[q] = (i < no) ? a.Qm[(int64_t)i * n + r] : 0.0;
  }
  double* mcol = a.Mm + (int64_t)r * t;
  for (int i = no - 1; i >= 0; --i) {
    const int qi = i >> 6;
    double yq = y[0];
#pragma unroll
    for (int q = 1; q < EY; ++q)
      if (q == qi) yq = y[q];
    const double yi = readlane_f64(yq, i & 63);
    const int ci = i * (i + 1) / 2;
    const double rii = rp[ci + i];
    const double xi = (fabs(rii) > tol) ? yi / rii : 0.0;
#pragma unroll
    for (int q = 0; q < EY; ++q) {
      const int k = lane + 64 * q;
      if (k < i) y[q] = fma(-xi, rp[ci + k], y[q]);
    }
    if (lane == 0) mcol[i] = xi;
  }
}

__device__ __forceinline__ void alg4_pgemm_body(const UpdArgs& a, const Blk bk) {
  __shared__ double red[4 * 16 * 64];
  __shared__ int occ[kMaxT];
  const int n = a.ell, t = a.t;
  const int no = min(a.sc->n_occ, n);
  const int nmt = (t + 31) / 32;
  const int mt = bk.x % nmt, ct = bk.x / nmt;
  const int m0 = 32 * mt, n0 = 32 * ct;
  const int64_t nobs = a.n_obs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (mt == 0) {
    // rows of empty slots are zero
    for (int sl = tid; sl < t; sl += 256) occ[sl] = 0;
    __syncthreads();
    for (int i = tid; i < no; i += 256) occ[a.sc->occ_slot[i]] = 1;
    __syncthreads();
    for (int idx = tid; idx < 32 * t; idx += 256) {
      const int sl = idx % t, c = n0 + idx / t;
      if (!occ[sl] && c < nobs) a.P[(int64_t)c * t + sl] = 0.0;
    }
  }
  if (m0 >= no) return;
  const double* M = a.Mm;
  const double* S = a.S;
  double out[2][2][4];
  gemm32_f64(m0, n0, n,
             [&](int m, int k) { return (m < no && k < n) ? M[(int64_t)k * t + m] : 0.0; },
             [&](int k, int c) { return (k < n && c < nobs) ? S[(int64_t)c * n + k] : 0.0; }, out, red);
  if (wave == 0) {
    const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + 16 * x + k4 + 4 * v, c = n0 + 16 * y + i16;
          if (m < no && c < nobs) a.P[(int64_t)c * t + a.sc->occ_slot[m]] = out[x][y][v];
        }
  }
}

// Y = S P^T (l x t) and P P^T (t x t) on the matrix cores: blocks [0, tY)
// take the tiles of Y, the rest those of P P^T.
__device__ __forceinline__ void hutch_gemm_body(const UpdArgs& a, const Blk bk) {
  __shared__ double red[4 * 16 * 64];
  const int n = a.ell, t = a.t;
  const int64_t nobs = a.n_obs;
  const int K = (int)nobs;
  const int tyM = (n + 31) / 32, tyN = (t + 31) / 32;
  const int tY = tyM * tyN;
  const double* S = a.S;
  const double* P = a.P;
  double out[2][2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  if (bk.x < tY) {
    const int m0 = 32 * (bk.x % tyM), n0 = 32 * (bk.x / tyM);
    gemm32_f64(m0, n0, K, [&](int r, int c) { return (r < n && c < K) ? S[(int64_t)c * n + r] : 0.0; },
               [&](int c, int j) { return (c < K && j < t) ? P[(int64_t)c * t + j] : 0.0; }, out, red);
    if (wave == 0)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = m0 + 16 * x + k4 + 4 * v, j = n0 + 16 * y + i16;
            if (r < n && j < t) a.Y[(int64_t)j * n + r] = out[x][y][v];
          }
  } else {
    const int b = bk.x - tY;
    const int m0 = 32 * (b % tyN), n0 = 32 * (b / tyN);
    gemm32_f64(m0, n0, K, [&](int i, int c) { return (i < t && c < K) ? P[(int64_t)c * t + i] : 0.0; },
               [&](int c, int j) { return (c < K && j < t) ? P[(int64_t)c * t + j] : 0.0; }, out, red);
    if (wave == 0)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = m0 + 16 * x + k4 + 4 * v, j = n0 + 16 * y + i16;
            if (i < t && j < t) a.PPt[(int64_t)j * t + i] = out[x][y][v];
          }
  }
}

// The NA-Hutch++ products without P (t <= kAlg4Gemm): P has rows
// P(occupied, :) = M S and zero rows for empty slots, so Y = S P^T =
// (S S^T) M^T and P P^T = M Y, at O(l^2 t) flops instead of O(l t n_obs).
// Columns of Y and rows and columns of P P^T are slots; occi maps a slot to
// its row of M (-1: empty).
__device__ __forceinline__ void hutch_occ_index(const UpdArgs& a, int* occi) {
  const int t = a.t, no = min(a.sc->n_occ, a.ell);
  for (int sl = threadIdx.x; sl < t; sl += blockDim.x) occi[sl] = -1;
  __syncthreads();
  for (int i = threadIdx.x; i < no; i += blockDim.x) occi[a.sc->occ_slot[i]] = i;
  __syncthreads();
}

__device__ __forceinline__ void hutch_y_body(const UpdArgs& a, const Blk bk) {
  __shared__ double red[4 * 16 * 64];
  __shared__ int occi[kMaxT];
  const int n = a.ell, t = a.t;
  hutch_occ_index(a, occi);
  const int tyM = (n + 31) / 32;
  const int m0 = 32 * (bk.x % tyM), n0 = 32 * (bk.x / tyM);
  const double* SS = a.SSTu;
  const double* M = a.Mm;
  double out[2][2][4];
  gemm32_f64(m0, n0, n, [&](int r, int k) { return (r < n && k < n) ? SS[(int64_t)k * n + r] : 0.0; },
             [&](int k, int j) {
               const int o = (j < t) ? occi[j] : -1;
               return (o >= 0 && k < n) ? M[(int64_t)k * t + o] : 0.0;
             },
             out, red);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave == 0) {
    const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = m0 + 16 * x + k4 + 4 * v, j = n0 + 16 * y + i16;
          if (r < n && j < t) a.Y[(int64_t)j * n + r] = out[x][y][v];
        }
  }
}

__device__ __forceinline__ void hutch_ppt_body(const UpdArgs& a, const Blk bk) {
  __shared__ double red[4 * 16 * 64];
  __shared__ int occi[kMaxT];
  const int n = a.ell, t = a.t;
  hutch_occ_index(a, occi);
  const int tyN = (t + 31) / 32;
  const int m0 = 32 * (bk.x % tyN), n0 = 32 * (bk.x / tyN);
  const double* M = a.Mm;
  const double* Y = a.Y;
  double out[2][2][4];
  gemm32_f64(m0, n0, n,
             [&](int i, int r) {
               const int o = (i < t) ? occi[i] : -1;
               return (o >= 0 && r < n) ? M[(int64_t)r * t + o] : 0.0;
             },
             [&](int r, int j) { return (r < n && j < t) ? Y[(int64_t)j * n + r] : 0.0; }, out, red);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave == 0) {
    const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = m0 + 16 * x + k4 + 4 * v, j = n0 + 16 * y + i16;
          if (i < t && j < t) a.PPt[(int64_t)j * t + i] = out[x][y][v];
        }
  }
}

__global__ __launch_bounds__(256) void hutch_y_kernel(UpdArgs a) { hutch_y_body(a, own_block()); }
__global__ __launch_bounds__(256) void hutch_y_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) hutch_y_body(*p, bk);
}
__global__ __launch_bounds__(256) void hutch_ppt_kernel(UpdArgs a) { hutch_ppt_body(a, own_block()); }
__global__ __launch_bounds__(256) void hutch_ppt_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) hutch_ppt_body(*p, bk);
}

__global__ __launch_bounds__(64) void alg4_q_kernel(UpdArgs a) { alg4_q_body(a, own_block()); }
__global__ __launch_bounds__(64) void alg4_q_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) alg4_q_body(*p, bk);
}
__global__ __launch_bounds__(256) void alg4_m_kernel(UpdArgs a) { alg4_m_body(a, own_block()); }
__global__ __launch_bounds__(256) void alg4_m_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) alg4_m_body(*p, bk);
}
__global__ __launch_bounds__(256) void alg4_pgemm_kernel(UpdArgs a) { alg4_pgemm_body(a, own_block()); }
__global__ __launch_bounds__(256) void alg4_pgemm_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) alg4_pgemm_body(*p, bk);
}
__global__ __launch_bounds__(256) void hutch_gemm_kernel(UpdArgs a) { hutch_gemm_body(a, own_block()); }
__global__ __launch_bounds__(256) void hutch_gemm_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) hutch_gemm_body(*p, bk);
}

// ---------------------------------------------------------------------------
// NA-Hutch++ (Alg. 8): the products of its small part, one thread per output
// entry (Y = S P^T and P P^T come from hutch_gemm_kernel).
// Stage 0: S_J gather.  Stage 1: K^T = (Y1 SJ2^T)^T, YG = Y1 G, A1 = Y1 SJ3^T,
// A2 = SJ3 Y2^T.  Stage 2: X = YG Y2^T, AA = A1 A2.
struct HutchWork {
  double *KT, *X, *AA, *YG, *A1, *A2, *SJ;
};

// K^T, X, AA, A1 and A2 are products of two of n1, n2, n3 (pairwise sums
// below l, so each holds fewer than l^2 / 4 entries); YG and S_J hold at most
// l t.  The layout follows the stream's l and t (hutch_work_doubles).
__device__ __forceinline__ HutchWork hutch_work(const UpdArgs& a) {
  const int64_t e4 = hutch_work_quarter(a.ell), et = (int64_t)a.ell * a.t;
  HutchWork w;
  w.KT = a.hw;
  w.X = w.KT + e4;
  w.AA = w.X + e4;
  w.YG = w.AA + e4;
  w.A1 = w.YG + et;
  w.A2 = w.A1 + e4;
  w.SJ = w.A2 + e4;
  return w;
}

__device__ __forceinline__ void hutch_mid_body(const UpdArgs& a, const Blk bk, int stage) {
  const int n = a.ell, t = a.t, n1 = a.n1, n2 = a.n2, n3 = a.ell - a.n1 - a.n2;
  const HutchWork w = hutch_work(a);
  const double* Y = a.Y;
  int64_t idx = (int64_t)bk.x * blockDim.x + threadIdx.x;
  if (stage == 0) {
    if (idx < (int64_t)n * t) {
      const int j = (int)(idx / n), r = (int)(idx % n);
      const int64_t Jj = a.J[j];
      w.SJ[idx] = (Jj >= 0) ? a.S[Jj * n + r] : 0.0;
    }
    return;
  }
  if (stage == 1) {
    const int64_t nK = (int64_t)n1 * n2, nYG = (int64_t)n1 * t, nA1 = (int64_t)n1 * n3, nA2 = (int64_t)n3 * n2;
    if (idx < nK) {
      const int b = (int)(idx % n2), aa = (int)(idx / n2);
      double s = 0.0;
      for (int j = 0; j < t; ++j) s = fma(Y[(int64_t)j * n + aa], w.SJ[(int64_t)j * n + n1 + b], s);
      w.KT[(int64_t)aa * n2 + b] = s;
      return;
    }
    idx -= nK;
    if (idx < nYG) {
      const int aa = (int)(idx % n1), j = (int)(idx / n1);
      double s = 0.0;
      for (int i = 0; i < t; ++i) s = fma(Y[(int64_t)i * n + aa], a.G[(int64_t)j * t + i], s);
      w.YG[(int64_t)j * n1 + aa] = s;
      return;
    }
    idx -= nYG;
    if (idx < nA1) {
      const int aa = (int)(idx % n1), c = (int)(idx / n1);
      double s = 0.0;
      for (int j = 0; j < t; ++j) s = fma(Y[(int64_t)j * n + aa], w.SJ[(int64_t)j * n + n1 + n2 + c], s);
      w.A1[(int64_t)c * n1 + aa] = s;
      return;
    }
    idx -= nA1;
    if (idx < nA2) {
      const int c = (int)(idx % n3), b = (int)(idx / n3);
      double s = 0.0;
      for (int j = 0; j < t; ++j) s = fma(w.SJ[(int64_t)j * n + n1 + n2 + c], Y[(int64_t)j * n + n1 + b], s);
      w.A2[(int64_t)b * n3 + c] = s;
    }
    return;
  }
  // X and AA row-major (row aa contiguous), for the reflector sweeps of the small kernel
  if (idx < (int64_t)n1 * n2) {
    const int b = (int)(idx % n2), aa = (int)(idx / n2);
    double s = 0.0;
    for (int j = 0; j < t; ++j) s = fma(w.YG[(int64_t)j * n1 + aa], Y[(int64_t)j * n + n1 + b], s);
    w.X[(int64_t)aa * n2 + b] = s;
    double s2 = 0.0;
    for (int c = 0; c < n3; ++c) s2 = fma(w.A1[(int64_t)c * n1 + aa], w.A2[(int64_t)b * n3 + c], s2);
    w.AA[(int64_t)aa * n2 + b] = s2;
  }
}

__global__ void hutch_mid_kernel(UpdArgs a, int stage) { hutch_mid_body(a, own_block(), stage); }

__global__ void hutch_mid_kernel_b(Batched<UpdArgs> L, int stage) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) hutch_mid_body(*p, bk, stage);
}

// The small part of Alg. 8 in one workgroup.  With the row blocks
// [0,n1), [n1,n1+n2), [n1+n2,l) of S, of S_J = Omega A_J and of Y:
//   K = Y1 SJ2^T, X = Y1 G Y2^T, A1 = Y1 SJ3^T, A2 = SJ3 Y2^T,
//   term1 = tr(K^+ X), corr = tr(K^+ A1 A2), h = <Y3, SJ3>, gpp = <G, P P^T>.
// K^+ is applied through a column-pivoted Householder QR of K^T truncated to
// its numerical rank r (max(n1, n2) eps |R_00|): K^- = Q_r R11^{-T} [I 0] Pi^T,
// the pseudo-inverse when K has full row rank.  With Z = rows Pi_r of X Q_r,
// tr(K^- X) = tr(R11^{-T} Z) = <R11^{-1}, Z>_F; R11^{-1} is formed in LDS.
__device__ __forceinline__ void hutch_small_body(const UpdArgs& a, const Blk bk) {
  constexpr int kMaxN1 = kMaxEll / 4;
  __shared__ double red[16];
  __shared__ double v[kMaxEll];
  __shared__ double cn[kMaxN1];
  __shared__ int perm[kMaxN1];
  __shared__ double rinv[kMaxN1 * kMaxN1];
  const int n = a.ell, t = a.t, n1 = a.n1, n2 = a.n2, n3 = a.ell - a.n1 - a.n2;
  const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nth >> 6;
  rid_update* rec = a.recs + a.u;
  const double F = a.Fu[a.u];
  // work layout: KT n2 x n1 (column-major, ld n2), X and AA n1 x n2 (row-major), SJ l x t
  const HutchWork hwk = hutch_work(a);
  double* KT = hwk.KT;
  double* X = hwk.X;
  double* AA = hwk.AA;
  const double* SJ = hwk.SJ;
  const double* Y = a.Y;
  const double* G = a.G;
  // h and gpp
  double hp = 0.0, gp = 0.0;
  for (int64_t idx = tid; idx < (int64_t)n3 * t; idx += nth) {
    const int c = (int)(idx % n3), j = (int)(idx / n3);
    hp = fma(Y[(int64_t)j * n + n1 + n2 + c], SJ[(int64_t)j * n + n1 + n2 + c], hp);
  }
  for (int64_t idx = tid; idx < (int64_t)t * t; idx += nth) gp = fma(G[idx], a.PPt[idx], gp);
  const double h = block_sum(hp, red);
  const double gpp = block_sum(gp, red);
  double term1 = 0.0, corr = 0.0;
  int trunc = 0;
  if (n1 > 0 && n2 > 0) {
    for (int i = tid; i < n1; i += nth) perm[i] = i;
    __syncthreads();
    // column-pivoted Householder QR of KT (n2 x n1)
    int rank = 0;
    double r00 = 0.0;
    const int nsteps = min(n1, n2);
    for (int jj = 0; jj < nsteps; ++jj) {
      // squared norms of the remaining columns, rows jj..n2-1 (recomputed)
      for (int c = jj + wv; c < n1; c += nw) {
        const double* col = KT + (int64_t)c * n2;
        double s = 0.0;
        for (int i = jj + lane; i < n2; i += 64) s = fma(col[i], col[i], s);
        s = wave_sum(s);
        if (lane == 0) cn[c] = s;
      }
      __syncthreads();
      // pivot: the first column of largest norm, found by every wave
      int piv = n1;
      double best = -1.0;
      for (int c = jj + lane; c < n1; c += 64)
        if (cn[c] > best) {
          best = cn[c];
          piv = c;
        }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int op = __shfl_xor(piv, off);
        if (ob > best || (ob == best && op < piv)) {
          best = ob;
          piv = op;
        }
      }
      if (jj == 0) r00 = sqrt(best);
      if (!(sqrt(best) > (double)max(n1, n2) * 2.220446049250313e-16 * r00) || best == 0.0) break;
      if (piv != jj) {
        for (int i = tid; i < n2; i += nth) {
          const double tmp = KT[(int64_t)jj * n2 + i];
          KT[(int64_t)jj * n2 + i] = KT[(int64_t)piv * n2 + i];
          KT[(int64_t)piv * n2 + i] = tmp;
        }
        __syncthreads();
        if (tid == 0) {
          const int tp = perm[jj];
          perm[jj] = perm[piv];
          perm[piv] = tp;
        }
      }
      double* x = KT + (int64_t)jj * n2 + jj;
      const int len = n2 - jj;
      double part = 0.0;
      for (int i = 1 + tid; i < len; i += nth) part += x[i] * x[i];
      const double xn2 = block_sum(part, red);
      const double alpha = x[0];
      double tau = 0.0, beta = alpha;
      if (xn2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);
        for (int i = tid; i < len; i += nth) v[i] = (i == 0) ? 1.0 : x[i] * scal;
      } else {
        for (int i = tid; i < len; i += nth) v[i] = (i == 0) ? 1.0 : 0.0;
      }
      __syncthreads();
      for (int i = 1 + tid; i < len; i += nth) x[i] = v[i];
      if (tid == 0) x[0] = beta;
      if (tau != 0.0) {
        for (int c = jj + 1 + wv; c < n1; c += nw) {
          double* y = KT + (int64_t)c * n2 + jj;
          double s = 0.0;
          for (int i = lane; i < len; i += 64) s = fma(v[i], y[i], s);
          const double g = tau * wave_sum(s);
          for (int i = lane; i < len; i += 64) y[i] -= g * v[i];
        }
        // rows of X and AA: x^T <- x^T H
        for (int rr = wv; rr < 2 * n1; rr += nw) {
          double* row = ((rr < n1) ? X + (int64_t)rr * n2 : AA + (int64_t)(rr - n1) * n2) + jj;
          double s = 0.0;
          for (int i = lane; i < len; i += 64) s = fma(v[i], row[i], s);
          const double g = tau * wave_sum(s);
          for (int i = lane; i < len; i += 64) row[i] -= g * v[i];
        }
      }
      __syncthreads();
      ++rank;
    }
    trunc = (rank < n1);
    // R11^{-1} (upper triangular, row-major in LDS), rows from the bottom:
    // Rinv(i, j) = (delta_ij - sum_{i<k<=j} R(i, k) Rinv(k, j)) / R(i, i),
    // R(i, k) = KT[k n2 + i].  Eight lanes per entry j.
    const int r = rank;
    for (int i = r - 1; i >= 0; --i) {
      for (int k = i + tid; k < r; k += nth) v[k] = KT[(int64_t)k * n2 + i];
      __syncthreads();
      const double rii = v[i];
      const int j = i + (tid >> 3), q = tid & 7;
      double s = 0.0;
      if (j < r)
        for (int k = i + 1 + q; k <= j; k += 8) s = fma(v[k], rinv[k * r + j], s);
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      if (j < r && q == 0) rinv[i * r + j] = ((j == i ? 1.0 : 0.0) - s) / rii;
      __syncthreads();
    }
    // term1 = <R11^{-1}, Z_X>, corr = <R11^{-1}, Z_AA>, Z(i, j) = M(perm[i], j)
    double tr_x = 0.0, tr_a = 0.0;
    for (int idx = tid; idx < r * r; idx += nth) {
      const int i = idx / r, j = idx % r;
      if (j < i) continue;
      const double ri = rinv[idx];
      tr_x = fma(ri, X[(int64_t)perm[i] * n2 + j], tr_x);
      tr_a = fma(ri, AA[(int64_t)perm[i] * n2 + j], tr_a);
    }
    term1 = block_sum(tr_x, red);
    corr = block_sum(tr_a, red);
  }
  if (tid == 0) {
    const double tr_est = term1 + (h - corr) / n3;
    const double E2 = F - 2.0 * tr_est + gpp;
    rec->E2 = E2;
    rec->tr_est = tr_est;
    rec->gpp = gpp;
    rec->term1 = term1;
    rec->h = h;
    rec->corr = corr;
    if (trunc) rec->flags |= RID_UPD_PINV_TRUNCATED;
  }
}

__global__ __launch_bounds__(1024) void hutch_small_kernel(UpdArgs a) { hutch_small_body(a, own_block()); }

__global__ __launch_bounds__(1024) void hutch_small_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) hutch_small_body(*p, bk);
}

// The same small phase with K^T, X and AA held in registers.  The n1 columns
// of K^T and the 2 n1 rows of X and AA are vectors of length n2; vector q
// lives in wave q % NW (slot q / NW), element r in lane r % 64 (e = r / 64).
// Step jj of the pivoted QR: every wave writes the remaining norms of its
// K^T vectors to LDS; one barrier; every wave finds the pivot; its owner forms
// the reflector and publishes it; one barrier; every wave applies it to its
// unchosen K^T vectors and to all X / AA vectors.  Vectors are never swapped:
// pos[i] is the K^T column chosen at step i.
template <int E, int NS, int NW>
__device__ __forceinline__ void hutch_small_reg_body(const UpdArgs& a, const Blk bk) {
  constexpr int kMaxN1 = kMaxEll / 4;
  __shared__ double red[16];
  __shared__ double vb[2][64 * E];
  __shared__ double tb[2];
  __shared__ double cn[kMaxN1];
  __shared__ double cref[kMaxN1];
  __shared__ int pos[kMaxN1];
  __shared__ int ipos[kMaxN1];
  __shared__ double rinv[kMaxN1 * kMaxN1];
  __shared__ double qred[NW][4 * 64];   // each wave's dot sums (wave_sum4)
  const int n = a.ell, t = a.t, n1 = a.n1, n2 = a.n2, n3 = a.ell - a.n1 - a.n2;
  const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6;
  rid_update* rec = a.recs + a.u;
  const double F = a.Fu[a.u];
  const HutchWork hwk = hutch_work(a);
  const double* Y = a.Y;
  const double* G = a.G;
  // h and gpp
  double hp = 0.0, gp = 0.0;
  for (int64_t idx = tid; idx < (int64_t)n3 * t; idx += nth) {
    const int c = (int)(idx % n3), j = (int)(idx / n3);
    hp = fma(Y[(int64_t)j * n + n1 + n2 + c], hwk.SJ[(int64_t)j * n + n1 + n2 + c], hp);
  }
  for (int64_t idx = tid; idx < (int64_t)t * t; idx += nth) gp = fma(G[idx], a.PPt[idx], gp);
  const double h = block_sum(hp, red);
  const double gpp = block_sum(gp, red);
  // vectors: [0, n1) columns of K^T, [n1, 2 n1) rows of X, [2 n1, 3 n1) rows of AA
  const int nv = 3 * n1;
  double vec[NS][E];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int q = wave + NW * sl;
    const double* src = nullptr;
    if (q < n1) src = hwk.KT + (int64_t)q * n2;
    else if (q < 2 * n1) src = hwk.X + (int64_t)(q - n1) * n2;
    else if (q < nv) src = hwk.AA + (int64_t)(q - 2 * n1) * n2;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int r = lane + 64 * e;
      vec[sl][e] = (src && r < n2) ? src[r] : 0.0;
    }
  }
  for (int i = tid; i < n1; i += nth) ipos[i] = -1;
  __syncthreads();
  int rank = 0;
  double r00 = 0.0;
  const int nsteps = min(n1, n2);
  // Squared norms (rows jj..) of the K^T vectors in LDS (cn; -1 once
  // chosen), downdated after each step by the square of the vector's element
  // jj; recomputed when the downdate has cancelled below sqrt(eps) of the
  // norm it started from (cref), as in LAPACK's column-pivoted QR.  Slots
  // below nsk hold K^T vectors.
  const int nsk = (n1 + NW - 1) / NW;
  auto norm_rows = [&](int sl, int from) {
    double part = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int r = lane + 64 * e;
      if (r >= from && r < n2) part = fma(vec[sl][e], vec[sl][e], part);
    }
    return wave_sum(part);
  };
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int q = wave + NW * sl;
    if (sl < nsk && q < n1) {
      const double c0 = norm_rows(sl, 0);
      if (lane == 0) {
        cn[q] = c0;
        cref[q] = c0;
      }
    }
  }
  constexpr double kTol3z = 1.4901161193847656e-08;  // sqrt(2^-53 * 2)
  for (int jj = 0; jj < nsteps; ++jj) {
    const int buf = jj & 1;
    __syncthreads();
    // pivot: the first unchosen column of largest norm
    int piv = n1;
    double best = -1.0;
    for (int c = lane; c < n1; c += 64)
      if (cn[c] > best) {
        best = cn[c];
        piv = c;
      }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int op = __shfl_xor(piv, off);
      if (ob > best || (ob == best && op < piv)) {
        best = ob;
        piv = op;
      }
    }
    if (jj == 0) r00 = sqrt(best);
    if (!(sqrt(best) > (double)max(n1, n2) * 2.220446049250313e-16 * r00) || best <= 0.0) break;
    // reflector of the pivot vector (rows jj..n2-1), formed by its owner
    if (wave == piv % NW) {
      const int os = piv / NW;
      double x[E];
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] = 0.0;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        if (sl == os)
#pragma unroll
          for (int e = 0; e < E; ++e) x[e] = vec[sl][e];
      double part = 0.0, al = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = lane + 64 * e;
        if (r > jj && r < n2) part = fma(x[e], x[e], part);
        if (e == jj / 64) al = x[e];
      }
      const double xn2 = wave_sum(part);
      const double alpha = __shfl(al, jj & 63);
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xn2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = lane + 64 * e;
        const double vr = (r == jj) ? 1.0 : ((r > jj && r < n2) ? x[e] * scal : 0.0);
        vb[buf][r] = vr;
        if (r == jj) x[e] = beta;
        else if (r > jj) x[e] = vr;
      }
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        if (sl == os)
#pragma unroll
          for (int e = 0; e < E; ++e) vec[sl][e] = x[e];
      if (lane == 0) {
        tb[buf] = tau;
        pos[jj] = piv;
        ipos[piv] = jj;
        cn[piv] = -1.0;
      }
    }
    __syncthreads();
    const double tau = tb[buf];
    if (tau != 0.0) {
      double v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = lane + 64 * e;
        v[e] = (r >= jj && r < n2) ? vb[buf][r] : 0.0;
      }
      // Chosen pivots and empty slots take no reflector, and v is zero above
      // row jj: their dots, sums and row chunks wholly above jj are skipped
      // by scalar branches (the skipped terms are exact zeros).
      constexpr int B = 8;
      const int e0 = jj >> 6;
#pragma unroll
      for (int s0 = 0; s0 < NS; s0 += B) {
        if (wave + NW * s0 >= nv) continue;
        double d[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
          d[i] = 0.0;
          if (s0 + i < NS)
#pragma unroll
            for (int e = 0; e < E; ++e)
              if (e >= e0) d[i] = fma(v[e], vec[s0 + i][e], d[i]);
        }
#pragma unroll
        for (int h = 0; h < B; h += 4) {
          double d4[4] = {d[h], d[h + 1], d[h + 2], d[h + 3]};
          wave_sum4<4>(d4, qred[wave]);
#pragma unroll
          for (int u = 0; u < 4; ++u) d[h + u] = d4[u];
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
          if (s0 + i >= NS) continue;
          const int q = wave + NW * (s0 + i);
          const bool apply = (q < n1) ? (ipos[q] < 0) : (q < nv);
          if (apply) {
            const double g = tau * d[i];
#pragma unroll
            for (int e = 0; e < E; ++e)
              if (e >= e0) vec[s0 + i][e] = fma(-g, v[e], vec[s0 + i][e]);
          }
        }
      }
    }
    // downdate the norms of the unchosen K^T vectors to rows jj+1..
    {
      const int ej = jj >> 6, lj = jj & 63;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        const int q = wave + NW * sl;
        if (sl < nsk && q < n1 && ipos[q] < 0) {
          double xe = vec[sl][0];
#pragma unroll
          for (int e = 1; e < E; ++e)
            if (e == ej) xe = vec[sl][e];
          const double xj = readlane_f64(xe, lj);
          const double nn = cn[q] - xj * xj;
          if (nn <= kTol3z * cref[q]) {
            const double c1 = norm_rows(sl, jj + 1);
            if (lane == 0) {
              cn[q] = c1;
              cref[q] = c1;
            }
          } else if (lane == 0) {
            cn[q] = nn;
          }
        }
      }
    }
    ++rank;
  }
  const int r = rank;
  const int trunc = (rank < n1);
  double term1 = 0.0, corr = 0.0;
  if (r > 0) {
    // R11 (row-major r x r in LDS): R(i, k) = element i of K^T vector pos[k]
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int q = wave + NW * sl;
      if (q < n1) {
        const int k = ipos[q];
        if (k >= 0)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int i = lane + 64 * e;
            if (i <= k) rinv[i * r + k] = vec[sl][e];
          }
      }
    }
    __syncthreads();
    // in-place inverse, rows from the bottom: row i of R is read into
    // registers, then overwritten by row i of R^{-1}; eight lanes per entry
    constexpr int kPerPass = 64 * NW / 8;  // entries per pass
    for (int i = r - 1; i >= 0; --i) {
      const int qq = tid & 7;
      const double rii = rinv[i * r + i];
      double sum[kMaxN1 / kPerPass + 1];
#pragma unroll
      for (int ps = 0; ps * kPerPass < kMaxN1; ++ps) {
        const int j = i + ps * kPerPass + (tid >> 3);
        double sv = 0.0;
        if (j < r)
          for (int k = i + 1 + qq; k <= j; k += 8) sv = fma(rinv[i * r + k], rinv[k * r + j], sv);
        sv += __shfl_xor(sv, 1);
        sv += __shfl_xor(sv, 2);
        sv += __shfl_xor(sv, 4);
        sum[ps] = sv;
      }
      __syncthreads();
#pragma unroll
      for (int ps = 0; ps * kPerPass < kMaxN1; ++ps) {
        const int j = i + ps * kPerPass + (tid >> 3);
        if (j < r && qq == 0) rinv[i * r + j] = ((j == i ? 1.0 : 0.0) - sum[ps]) / rii;
      }
      __syncthreads();
    }
    // term1 = <R11^{-1}, Z_X>, corr = <R11^{-1}, Z_AA>, Z(i, j) = element j of
    // the X (AA) vector of row pos[i]
    double tx = 0.0, ta = 0.0;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int q = wave + NW * sl;
      if (q >= n1 && q < nv) {
        const int row = (q < 2 * n1) ? q - n1 : q - 2 * n1;
        const int i = ipos[row];
        if (i >= 0) {
          double part = 0.0;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int j = lane + 64 * e;
            if (j >= i && j < r) part = fma(rinv[i * r + j], vec[sl][e], part);
          }
          if (q < 2 * n1) tx += part;
          else ta += part;
        }
      }
    }
    term1 = block_sum(tx, red);
    corr = block_sum(ta, red);
  }
  if (tid == 0) {
    const double tr_est = term1 + (h - corr) / n3;
    const double E2 = F - 2.0 * tr_est + gpp;
    rec->E2 = E2;
    rec->tr_est = tr_est;
    rec->gpp = gpp;
    rec->term1 = term1;
    rec->h = h;
    rec->corr = corr;
    if (trunc) rec->flags |= RID_UPD_PINV_TRUNCATED;
  }
}

template <int E, int NS, int NW>
__global__ __launch_bounds__(64 * NW) void hutch_small_reg_kernel(UpdArgs a) { hutch_small_reg_body<E, NS, NW>(a, own_block()); }

template <int E, int NS, int NW>
__global__ __launch_bounds__(64 * NW) void hutch_small_reg_kernel_b(Batched<UpdArgs> L) {
  const UpdArgs* p;
  Blk bk;
  if (batched_block(L, p, bk)) hutch_small_reg_body<E, NS, NW>(*p, bk);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// SS^T, F and the ridge of every update of a batch (Alg. 3 steps 11, 13, 17-18)
hipError_t launch_update_batch(const BatchArgs& b, hipStream_t s) {
  const int nt = (b.ell + 31) / 32;
  hipLaunchKernelGGL(sst_batch_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, b);
  switch ((b.ell + 63) / 64) {
    case 1: hipLaunchKernelGGL(tridiag_kernel<1>, dim3(b.nz), dim3(1024), 0, s, b); break;
    case 2: hipLaunchKernelGGL(tridiag_kernel<2>, dim3(b.nz), dim3(1024), 0, s, b); break;
    case 3: hipLaunchKernelGGL(tridiag_kernel<3>, dim3(b.nz), dim3(1024), 0, s, b); break;
    case 4: hipLaunchKernelGGL(tridiag_kernel<4>, dim3(b.nz), dim3(1024), 0, s, b); break;
    case 5: hipLaunchKernelGGL(tridiag_kernel<5>, dim3(b.nz), dim3(1024), 0, s, b); break;
    case 6: hipLaunchKernelGGL(tridiag_kernel<6>, dim3(b.nz), dim3(1024), 0, s, b); break;
    case 7: hipLaunchKernelGGL(tridiag_kernel<7>, dim3(b.nz), dim3(1024), 0, s, b); break;
    default: hipLaunchKernelGGL(tridiag_kernel<8>, dim3(b.nz), dim3(1024), 0, s, b); break;
  }
  const int kk = std::min(b.k, b.ell);
  constexpr int per_wg = kEigWaves * 64 / kEigLanesStream;
  hipLaunchKernelGGL(tridiag_eig_kernel, dim3(b.nz, (kk + per_wg - 1) / per_wg), dim3(64 * kEigWaves), 0, s, b);
  hipLaunchKernelGGL(tridiag_ridge_kernel, dim3(b.nz), dim3(64), 0, s, b);
  return hipGetLastError();
}

// scores and selection (Alg. 3 steps 17-27)
hipError_t launch_update_q_all(const UpdArgs& a0, int nz, hipStream_t s) {
  with_em(a0.ell, [&](auto em) {
    hipLaunchKernelGGL((scores_q_all_kernel<decltype(em)::value>), dim3(a0.ell, nz), dim3(64), 0, s, a0);
  });
  return hipGetLastError();
}

hipError_t launch_update_select(const UpdArgs& a, hipStream_t s, bool with_q) {
  const int items = a.t + a.cnt;
  if (with_q)
    with_em(a.ell, [&](auto em) {
      hipLaunchKernelGGL((scores_q_kernel<decltype(em)::value>), dim3(a.ell), dim3(64), 0, s, a);
    });
  hipLaunchKernelGGL(scores_gemm_kernel, dim3(((a.ell + 31) / 32) * ((items + 31) / 32)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(scores_fin_kernel, dim3(items), dim3(64), 0, s, a);
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// new basis columns into the column pool and their Gram entries
hipError_t launch_update_gram(const UpdArgs& a, hipStream_t s) {
  if (a.data_f64) {
    const int tt = (a.t + kGramTile - 1) / kGramTile;
    hipLaunchKernelGGL(gram_kernel<double>, dim3(a.gslabs, tt, tt), dim3(1024), 0, s, a);
  } else if (a.gram_split) {
    const size_t lds = gram_split_lds(a.t);
    const void* f = gram_split_fn(a.t, false);
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {const_cast<UpdArgs*>(&a)};
    (void)hipLaunchKernel(f, dim3(a.gslabs, gram_split_groups(a.t)), dim3(64 * kGsWaves), args, lds, s);
  } else {
    const int tq = (a.t + 31) / 32;
    const int groups = (tq * tq + kGramGroup - 1) / kGramGroup;
    const size_t lds = (size_t)2 * gram_stage_cols(a.t) * kGramKC * sizeof(float) +
                       (size_t)gram_stage_cols(a.t) * sizeof(uint64_t) + (size_t)a.t * sizeof(int);
    static size_t attr_lds = 0;  // raised whenever a larger basis needs more
    if (lds > attr_lds) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(gram_f32_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr_lds = lds;
    }
    hipLaunchKernelGGL(gram_f32_kernel, dim3(a.gslabs, groups), dim3(64 * kGramWaves), lds, s, a);
  }
  hipLaunchKernelGGL(gram_zero_kernel, dim3(a.t), dim3(kMaxT), 0, s, a);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(a.t, (a.t + 63) / 64), dim3(64 * kGramReduceWaves), 0, s, a);
  if (!a.data_f64 && a.gram_split) {
    if (a.flush_last) hipLaunchKernelGGL(gram_pool_flush_kernel, dim3(kPoolFlushBlocks, a.t), dim3(256), 0, s, a);
    hipLaunchKernelGGL(gram_ptr_kernel, dim3(1), dim3(kMaxT), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_update_gram_run(const UpdArgs& a, int nu, int nq, int nj, const DevScalars* sc_hist,
                                  const int64_t* J_hist, GramRun* run, hipStream_t s) {
  hipLaunchKernelGGL(gram_run_list_kernel, dim3(1), dim3(256), 0, s, a, nu, sc_hist, J_hist, run);
  if (nq == 0) return hipGetLastError();
  UpdArgs g = a;
  g.grun = run;
  const int cols = std::max(nj, 1);
  const void* f = gram_split_fn(cols, false);
  const size_t lds = gram_split_lds(cols);
  (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  void* args[] = {&g};
  const int groups = (gsplit_tiles(nq, nj) + kGsGroup - 1) / kGsGroup;
  (void)hipLaunchKernel(f, dim3(a.gslabs, groups), dim3(64 * kGsWaves), args, lds, s);
  return hipGetLastError();
}

hipError_t launch_update_gram_run_entries(const UpdArgs& aw, int w, const GramRun* run, hipStream_t s) {
  UpdArgs g = aw;
  g.grun = run;
  g.grun_u = w;
  hipLaunchKernelGGL(gram_zero_kernel, dim3(aw.t), dim3(kMaxT), 0, s, aw);
  hipLaunchKernelGGL(gram_reduce_run_kernel, dim3(aw.t, kGramRunCols / 64), dim3(64 * kGramReduceWaves), 0, s, g);
  hipLaunchKernelGGL(gram_ptr_kernel, dim3(1), dim3(kMaxT), 0, s, aw);
  return hipGetLastError();
}

// Alg. 4 and Alg. 8
static void alg4_m_attributes() {
  static bool done = false;
  if (done) return;
  const int lds = (int)alg4_m_lds(kAlg4Gemm);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(alg4_m_kernel), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(alg4_m_kernel_b), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds);
  done = true;
}

hipError_t launch_update_coeff(const UpdArgs& a, hipStream_t s, bool want_p) {
  alg4_m_attributes();
  // Householder QR of Omega A_J: in registers when it fits, else through L2
  const int E = (a.ell + 63) / 64;
  if (E <= 1 && a.t <= 16)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<1, 2, 8>), dim3(1), dim3(512), 0, s, a);
  else if (E <= 2 && a.t <= 64)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<2, 8, 8>), dim3(1), dim3(512), 0, s, a);
  else if (E <= 4 && a.t <= 112)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<4, 14, 8>), dim3(1), dim3(512), 0, s, a);
  else if (E <= 5 && a.t <= 152)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<5, 19, 8>), dim3(1), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL(alg4_qr_kernel, dim3(1), dim3(1024), 0, s, a);
  if (a.t <= kAlg4Gemm) {
    hipLaunchKernelGGL(alg4_q_kernel, dim3(a.t), dim3(64), 0, s, a);
    hipLaunchKernelGGL(alg4_m_kernel, dim3((a.ell + 3) / 4), dim3(256), alg4_m_lds(a.t), s, a);
    if (want_p)
      hipLaunchKernelGGL(alg4_pgemm_kernel, dim3((unsigned)(((a.t + 31) / 32) * ((a.n_obs + 31) / 32))),
                         dim3(256), 0, s, a);
    const int ty = (a.ell + 31) / 32, tt = (a.t + 31) / 32;
    hipLaunchKernelGGL(hutch_y_kernel, dim3(ty * tt), dim3(256), 0, s, a);
    hipLaunchKernelGGL(hutch_ppt_kernel, dim3(tt * tt), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(alg4_apply_kernel, dim3((unsigned)a.n_obs), dim3(64), 0, s, a);
    const int tiles = ((a.ell + 31) / 32) * ((a.t + 31) / 32) + ((a.t + 31) / 32) * ((a.t + 31) / 32);
    hipLaunchKernelGGL(hutch_gemm_kernel, dim3(tiles), dim3(256), 0, s, a);
  }
  {
    const int n3 = a.ell - a.n1 - a.n2;
    const int64_t s0 = (int64_t)a.ell * a.t;
    const int64_t s1 = (int64_t)a.n1 * a.n2 + (int64_t)a.n1 * a.t + (int64_t)a.n1 * n3 + (int64_t)n3 * a.n2;
    const int64_t s2 = (int64_t)a.n1 * a.n2;
    hipLaunchKernelGGL(hutch_mid_kernel, dim3((unsigned)((s0 + 255) / 256)), dim3(256), 0, s, a, 0);
    hipLaunchKernelGGL(hutch_mid_kernel, dim3((unsigned)((s1 + 255) / 256)), dim3(256), 0, s, a, 1);
    hipLaunchKernelGGL(hutch_mid_kernel, dim3((unsigned)((s2 + 255) / 256)), dim3(256), 0, s, a, 2);
  }
  // the pivoted QR of K^T in registers when K^T, X and AA fit, else through L2
  {
    const int E = (a.n2 + 63) / 64, nv = 3 * a.n1;
    if (a.n1 > 0 && E <= 1 && nv <= 8 * 4)
      hipLaunchKernelGGL((hutch_small_reg_kernel<1, 4, 8>), dim3(1), dim3(512), 0, s, a);
    else if (a.n1 > 0 && E <= 2 && nv <= 8 * 19)
      hipLaunchKernelGGL((hutch_small_reg_kernel<2, 19, 8>), dim3(1), dim3(512), 0, s, a);
    else if (a.n1 > 0 && E <= 3 && nv <= 8 * 29)
      hipLaunchKernelGGL((hutch_small_reg_kernel<3, 29, 8>), dim3(1), dim3(512), 0, s, a);
    else
      hipLaunchKernelGGL(hutch_small_kernel, dim3(1), dim3(1024), 0, s, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched planners: the same launches as above for several streams at once,
// one launch per kernel instance (streams needing another template instance
// of a kernel get a launch of their own)
// ---------------------------------------------------------------------------
namespace {

template <typename A>
struct Group {
  const void* func;
  size_t lds;
  std::vector<A> args;
  std::vector<int4> dims;
};

// Collects per-stream (kernel, grid) choices, then emits one launch per kernel.
template <typename A>
struct Planner {
  std::vector<Group<A>> groups;
  void add(const void* func, const A& a, int4 d, size_t lds = 0) {
    for (auto& g : groups)
      if (g.func == func) {
        g.args.push_back(a);
        g.dims.push_back(d);
        g.lds = std::max(g.lds, lds);
        return;
      }
    groups.push_back(Group<A>{func, lds, {a}, {d}});
  }
  int kind = 2;
  void emit(dim3 block, int extra, Stage& st, std::vector<BLaunch>& out) {
    for (auto& g : groups) {
      int maxb = 0;
      for (const int4& d : g.dims) maxb = std::max(maxb, d.x * d.y * d.z);
      if (maxb == 0) continue;
      BLaunch L{};
      L.func = g.func;
      L.grid = dim3((unsigned)maxb, (unsigned)g.args.size());
      L.block = block;
      L.lds = g.lds;
      L.args = st.put(g.args.data(), g.args.size());
      L.aux = st.put(g.dims.data(), g.dims.size());
      L.extra = extra;
      L.multi = false;
      L.kind = kind;
      out.push_back(L);
    }
    groups.clear();
  }
};

template <typename K>
const void* fn(K k) {
  return reinterpret_cast<const void*>(k);
}

}  // namespace

void plan_update_batch_b(const BatchArgs* h, int ns, Stage& st, std::vector<BLaunch>& out) {
  Planner<BatchArgs> P;
  for (int i = 0; i < ns; ++i) {
    const int nt = (h[i].ell + 31) / 32;
    P.add(fn(sst_batch_kernel_b), h[i], make_int4(nt * (nt + 1) / 2, 1, 1, 0));
  }
  P.emit(dim3(256), -1, st, out);
  // one workgroup per (stream, update); past one per compute unit the
  // workgroups go two to a unit at half the waves instead of in turns
  int total = 0, dev = 0, n_cu = 0;
  for (int i = 0; i < ns; ++i) total += h[i].nz;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    n_cu = 0;
  const bool half = n_cu > 0 && total > n_cu;
  for (int i = 0; i < ns; ++i) {
    const void* f;
#define RID_TRI(E) (half ? fn(tridiag_kernel_b<E, 8>) : fn(tridiag_kernel_b<E, 16>))
    switch ((h[i].ell + 63) / 64) {
      case 1: f = RID_TRI(1); break;
      case 2: f = RID_TRI(2); break;
      case 3: f = RID_TRI(3); break;
      case 4: f = RID_TRI(4); break;
      case 5: f = RID_TRI(5); break;
      case 6: f = RID_TRI(6); break;
      case 7: f = RID_TRI(7); break;
      default: f = RID_TRI(8); break;
    }
#undef RID_TRI
    P.add(f, h[i], make_int4(h[i].nz, 1, 1, 0));
  }
  P.emit(dim3(half ? 512 : 1024), -1, st, out);
  for (int i = 0; i < ns; ++i) {
    const int kk = std::min(h[i].k, h[i].ell);
    constexpr int per_wg = kEigWaves * 64 / kEigLanesBatch;
    P.add(fn(tridiag_eig_kernel_b), h[i], make_int4(h[i].nz, (kk + per_wg - 1) / per_wg, 1, 0));
  }
  P.emit(dim3(64 * kEigWaves), -1, st, out);
  for (int i = 0; i < ns; ++i) P.add(fn(tridiag_ridge_kernel_b), h[i], make_int4(h[i].nz, 1, 1, 0));
  P.emit(dim3(64), -1, st, out);
}

void plan_update_q_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out) {
  Planner<UpdArgs> P;
  for (int i = 0; i < ns; ++i)
    with_em(h[i].ell, [&](auto em) {
      P.add(fn(scores_q_kernel_b<decltype(em)::value>), h[i], make_int4(h[i].ell, 1, 1, 0));
    });
  P.emit(dim3(64), -1, st, out);
}

void plan_update_select_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out, bool with_q) {
  Planner<UpdArgs> P;
  if (with_q) plan_update_q_b(h, ns, st, out);
  for (int i = 0; i < ns; ++i) {
    const int items = h[i].t + h[i].cnt;
    P.add(fn(scores_gemm_kernel_b), h[i], make_int4(((h[i].ell + 31) / 32) * ((items + 31) / 32), 1, 1, 0));
  }
  P.emit(dim3(256), -1, st, out);
  for (int i = 0; i < ns; ++i) P.add(fn(scores_fin_kernel_b), h[i], make_int4(h[i].t + h[i].cnt, 1, 1, 0));
  P.emit(dim3(64), -1, st, out);
  for (int i = 0; i < ns; ++i) P.add(fn(select_kernel_b), h[i], make_int4(1, 1, 1, 0));
  P.emit(dim3(64), -1, st, out);
}

void plan_update_gram_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out) {
  Planner<UpdArgs> P64, P32, PS;
  P64.kind = P32.kind = PS.kind = 3;
  for (int i = 0; i < ns; ++i) {
    const UpdArgs& a = h[i];
    if (a.data_f64) {
      const int tt = (a.t + kGramTile - 1) / kGramTile;
      P64.add(fn(gram_kernel_b<double>), a, make_int4(a.gslabs, tt, tt, 0));
    } else if (a.gram_split) {
      PS.add(gram_split_fn(a.t, true), a, make_int4(a.gslabs, gram_split_groups(a.t), 1, 0), gram_split_lds(a.t));
    } else {
      const int tq = (a.t + 31) / 32;
      const int groups = (tq * tq + kGramGroup - 1) / kGramGroup;
      const size_t lds = (size_t)2 * gram_stage_cols(a.t) * kGramKC * sizeof(float) +
                         (size_t)gram_stage_cols(a.t) * sizeof(uint64_t) + (size_t)a.t * sizeof(int);
      P32.add(fn(gram_f32_kernel_b), a, make_int4(a.gslabs, groups, 1, 0), lds);
    }
  }
  P64.emit(dim3(1024), -1, st, out);
  static size_t attr_lds = 0;
  for (auto& g : P32.groups)
    if (g.lds > attr_lds) {
      (void)hipFuncSetAttribute(fn(gram_f32_kernel_b), hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds);
      attr_lds = g.lds;
    }
  P32.emit(dim3(64 * kGramWaves), -1, st, out);
  for (auto& g : PS.groups)
    (void)hipFuncSetAttribute(g.func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds);
  PS.emit(dim3(64 * kGsWaves), -1, st, out);
  Planner<UpdArgs> P;
  for (int i = 0; i < ns; ++i) P.add(fn(gram_zero_kernel_b), h[i], make_int4(h[i].t, 1, 1, 0));
  P.emit(dim3(kMaxT), -1, st, out);
  for (int i = 0; i < ns; ++i) P.add(fn(gram_reduce_kernel_b), h[i], make_int4(h[i].t, (h[i].t + 63) / 64, 1, 0));
  P.emit(dim3(64 * kGramReduceWaves), -1, st, out);
  for (int i = 0; i < ns; ++i)
    if (!h[i].data_f64 && h[i].gram_split && h[i].flush_last)
      P.add(fn(gram_pool_flush_kernel_b), h[i], make_int4(kPoolFlushBlocks, h[i].t, 1, 0));
  P.emit(dim3(256), -1, st, out);
  for (int i = 0; i < ns; ++i)
    if (!h[i].data_f64 && h[i].gram_split) P.add(fn(gram_ptr_kernel_b), h[i], make_int4(1, 1, 1, 0));
  P.emit(dim3(kMaxT), -1, st, out);
}

void plan_update_coeff_b(const UpdArgs* h, int ns, Stage& st, std::vector<BLaunch>& out, const bool* want_p) {
  alg4_m_attributes();
  const int4 one = make_int4(1, 1, 1, 0);
  {
    Planner<UpdArgs> Preg, Pl2;
    for (int i = 0; i < ns; ++i) {
      const UpdArgs& a = h[i];
      const int E = (a.ell + 63) / 64;
      if (E <= 1 && a.t <= 16) Preg.add(fn(alg4_qr_reg_kernel_b<1, 2, 8>), a, one);
      else if (E <= 2 && a.t <= 64) Preg.add(fn(alg4_qr_reg_kernel_b<2, 8, 8>), a, one);
      else if (E <= 4 && a.t <= 112) Preg.add(fn(alg4_qr_reg_kernel_b<4, 14, 8>), a, one);
      else if (E <= 5 && a.t <= 152) Preg.add(fn(alg4_qr_reg_kernel_b<5, 19, 8>), a, one);
      else Pl2.add(fn(alg4_qr_kernel_b), a, one);
    }
    Preg.emit(dim3(512), -1, st, out);
    Pl2.emit(dim3(1024), -1, st, out);
  }
  Planner<UpdArgs> P;
  for (int i = 0; i < ns; ++i)
    if (h[i].t <= kAlg4Gemm) P.add(fn(alg4_q_kernel_b), h[i], make_int4(h[i].t, 1, 1, 0));
  P.emit(dim3(64), -1, st, out);
  for (int i = 0; i < ns; ++i)
    if (h[i].t <= kAlg4Gemm)
      P.add(fn(alg4_m_kernel_b), h[i], make_int4((h[i].ell + 3) / 4, 1, 1, 0), alg4_m_lds(h[i].t));
  P.emit(dim3(256), -1, st, out);
  for (int i = 0; i < ns; ++i)
    if (h[i].t <= kAlg4Gemm && (!want_p || want_p[i]))
      P.add(fn(alg4_pgemm_kernel_b), h[i],
            make_int4((int)(((h[i].t + 31) / 32) * ((h[i].n_obs + 31) / 32)), 1, 1, 0));
  P.emit(dim3(256), -1, st, out);
  for (int i = 0; i < ns; ++i)
    if (h[i].t > kAlg4Gemm) P.add(fn(alg4_apply_kernel_b), h[i], make_int4((int)h[i].n_obs, 1, 1, 0));
  P.emit(dim3(64), -1, st, out);
  // Y and P P^T: from S S^T and M, or from P above kAlg4Gemm
  for (int i = 0; i < ns; ++i) {
    const int ty = (h[i].ell + 31) / 32, tt = (h[i].t + 31) / 32;
    if (h[i].t <= kAlg4Gemm) P.add(fn(hutch_y_kernel_b), h[i], make_int4(ty * tt, 1, 1, 0));
    else P.add(fn(hutch_gemm_kernel_b), h[i], make_int4(ty * tt + tt * tt, 1, 1, 0));
  }
  P.emit(dim3(256), -1, st, out);
  for (int i = 0; i < ns; ++i) {
    const int tt = (h[i].t + 31) / 32;
    if (h[i].t <= kAlg4Gemm) P.add(fn(hutch_ppt_kernel_b), h[i], make_int4(tt * tt, 1, 1, 0));
  }
  P.emit(dim3(256), -1, st, out);
  for (int stage = 0; stage < 3; ++stage) {
    for (int i = 0; i < ns; ++i) {
      const UpdArgs& a = h[i];
      const int n3 = a.ell - a.n1 - a.n2;
      int64_t sz;
      if (stage == 0) sz = (int64_t)a.ell * a.t;
      else if (stage == 1) sz = (int64_t)a.n1 * a.n2 + (int64_t)a.n1 * a.t + (int64_t)a.n1 * n3 + (int64_t)n3 * a.n2;
      else sz = (int64_t)a.n1 * a.n2;
      P.add(fn(hutch_mid_kernel_b), a, make_int4((int)((sz + 255) / 256), 1, 1, 0));
    }
    P.emit(dim3(256), stage, st, out);
  }
  {
    Planner<UpdArgs> Preg, Pl2;
    for (int i = 0; i < ns; ++i) {
      const UpdArgs& a = h[i];
      const int E = (a.n2 + 63) / 64, nv = 3 * a.n1;
      if (a.n1 > 0 && E <= 1 && nv <= 8 * 4) Preg.add(fn(hutch_small_reg_kernel_b<1, 4, 8>), a, one);
      else if (a.n1 > 0 && E <= 2 && nv <= 8 * 19) Preg.add(fn(hutch_small_reg_kernel_b<2, 19, 8>), a, one);
      else if (a.n1 > 0 && E <= 3 && nv <= 8 * 29) Preg.add(fn(hutch_small_reg_kernel_b<3, 29, 8>), a, one);
      else Pl2.add(fn(hutch_small_kernel_b), a, one);
    }
    Preg.emit(dim3(512), -1, st, out);
    Pl2.emit(dim3(1024), -1, st, out);
  }
}

hipError_t run_launches(const std::vector<BLaunch>& v, hipStream_t s) {
  for (const BLaunch& L : v) {
    hipError_t e;
    if (L.multi) {
      MultiSketch ms{reinterpret_cast<const SketchArgs*>(L.args), reinterpret_cast<const int*>(L.aux), L.ns,
                     L.total};
      void* params[] = {&ms};
      e = hipLaunchKernel(L.func, L.grid, L.block, params, L.lds, s);
    } else {
      Batched<char> b{reinterpret_cast<const char*>(L.args), reinterpret_cast<const int4*>(L.aux)};
      int extra = L.extra;
      void* params[] = {&b, &extra};
      e = hipLaunchKernel(L.func, L.grid, L.block, params, L.lds, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Copies the selection state the coefficient phase reads (the slot lists
// and counters, G) into the update's snapshot slots.
__global__ void snapshot_kernel(UpdArgs a, DevScalars* sc_out, double* g_out) {
  const int64_t tt = (int64_t)a.t * a.t;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < tt) g_out[i] = a.G[i];
  constexpr int nw = (int)(sizeof(DevScalars) / sizeof(int32_t));
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < nw; k += blockDim.x)
      reinterpret_cast<int32_t*>(sc_out)[k] = reinterpret_cast<const int32_t*>(a.sc)[k];
}

hipError_t launch_update_snapshot(const UpdArgs& a, DevScalars* sc_out, double* g_out, hipStream_t s) {
  const int64_t tt = (int64_t)a.t * a.t;
  hipLaunchKernelGGL(snapshot_kernel, dim3((unsigned)((tt + 255) / 256)), dim3(256), 0, s, a, sc_out, g_out);
  return hipGetLastError();
}

// The same copies for several updates (one table entry each).
__global__ void snapshot_kernel_b(Batched<SnapArgs> L) {
  const SnapArgs* p;
  Blk bk;
  if (!batched_block(L, p, bk)) return;
  const int64_t tt = (int64_t)p->t * p->t;
  const int64_t i = (int64_t)bk.x * blockDim.x + threadIdx.x;
  if (i < tt) p->g_out[i] = p->G[i];
  constexpr int nw = (int)(sizeof(DevScalars) / sizeof(int32_t));
  if (bk.x == 0)
    for (int k = threadIdx.x; k < nw; k += blockDim.x)
      reinterpret_cast<int32_t*>(p->sc_out)[k] = reinterpret_cast<const int32_t*>(p->sc)[k];
}

void plan_update_snapshot_b(const SnapArgs* h, int n, Stage& st, std::vector<BLaunch>& out) {
  Planner<SnapArgs> P;
  for (int i = 0; i < n; ++i)
    P.add(fn(snapshot_kernel_b), h[i], make_int4((int)(((int64_t)h[i].t * h[i].t + 255) / 256), 1, 1, 0));
  P.emit(dim3(256), -1, st, out);
}

// ---------------------------------------------------------------------------
// Algs. 5-7 and the best of four (Alg. 3's coefficient steps).
//
// Per update, after the Alg. 4 phase formed P4 and its NA-Hutch++ record:
//   Alg. 5  P5 = G^{-1} (Omega A_J)^T (Omega A_obs) / l over the occupied
//           slots: G = L L^T (Cholesky), M5 = L^{-T} L^{-1} S_J^T / l, P5 = M5 S;
//   Alg. 6  the previous kept P with the rows of replaced slots zeroed (Pz),
//           r_A = S - S_J Pz over the columns it covers, the new slots' part
//           of pinv(S_J) applied to r_A (the Alg. 4 factorisation of the new
//           slots alone), P6 = Pz + that;
//   Alg. 7  T = G^{-1} A_J^T A_{J_prev} (equal to R^+ Q^T A_{J_prev} for the QR
//           of A_J when A_J has full column rank, from the exact Grams: the
//           current one, the previous one and the new-by-pruned products
//           taken before the pool copy), P7 = T P_prev;
// the columns observed since the previous update take P4's coefficients in
// Algs. 6 and 7.  Each candidate's estimate comes from the same NA-Hutch++
// kernels (Y = S P^T and P P^T from P); the smallest E^2 wins, ties to the
// lowest q, and the kept P becomes the stream's P and the next update's P_prev.
// ---------------------------------------------------------------------------

// Pruned slots (occupied before the update, holding another column or none
// after it), in slot order, into LDS; returns their count.
__device__ int best4_pruned(const UpdArgs& a, const B4Args& b, int* pr) {
  __shared__ int cnt;
  if (threadIdx.x == 0) {
    int n = 0;
    for (int j = 0; j < a.t; ++j)
      if (b.J_prev[j] >= 0 && a.J[j] != b.J_prev[j]) pr[n++] = j;
    cnt = n;
  }
  __syncthreads();
  return cnt;
}

// New-by-pruned products over one Gram slab: tile (32 new, 32 pruned) of
// partial sums into gpart[slab][t][t] (compact indices).
template <typename T>
__global__ __launch_bounds__(256) void best4_cross_kernel(UpdArgs a, B4Args b) {
  __shared__ double red[4 * 16 * 64];
  __shared__ int pr[kMaxT];
  const int t = a.t;
  const int npr = best4_pruned(a, b, pr);
  const int nn = a.sc->n_new;
  const int tiles_n = (t + 31) / 32;
  const int it = blockIdx.x % tiles_n, jt = blockIdx.x / tiles_n;
  if (32 * it >= nn || 32 * jt >= npr) return;
  const int64_t r0 = (int64_t)blockIdx.y * a.gslab_rows;
  const int64_t r1 = min(a.m, r0 + a.gslab_rows);
  const int K = (int)max((int64_t)0, r1 - r0);
  const T* pool = reinterpret_cast<const T*>(a.cpool);
  double out[2][2][4];
  gemm32_f64(32 * it, 32 * jt, K,
             [&](int i, int k) {
               if (i >= nn || k >= K) return 0.0;
               const T* col = reinterpret_cast<const T*>(a.colptr[a.J[a.sc->new_slot[i]]]);
               return (double)col[r0 + k];
             },
             [&](int k, int j) {
               return (j < npr && k < K) ? (double)pool[(int64_t)pr[j] * a.ldc + r0 + k] : 0.0;
             },
             out, red);
  if ((threadIdx.x >> 6) == 0) {
    const int lane = threadIdx.x & 63, i16 = lane & 15, k4 = lane >> 4;
    double* part = a.gpart + (int64_t)blockIdx.y * t * t;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 32 * it + 16 * x + k4 + 4 * v, j = 32 * jt + 16 * y + i16;
          if (i < nn && j < npr) part[(int64_t)j * t + i] = out[x][y][v];
        }
  }
}

// Xc(new slot, pruned slot) = sum over the slabs in slab order.
__global__ __launch_bounds__(256) void best4_cross_reduce_kernel(UpdArgs a, B4Args b) {
  __shared__ int pr[kMaxT];
  const int t = a.t;
  const int npr = best4_pruned(a, b, pr);
  const int nn = a.sc->n_new;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nn * npr) return;
  const int i = (int)(idx % nn), j = (int)(idx / nn);
  double s = 0.0;
  for (int sl = 0; sl < a.gslabs; ++sl) s += a.gpart[(int64_t)sl * t * t + (int64_t)j * t + i];
  b.Xc[(int64_t)pr[j] * t + a.sc->new_slot[i]] = s;
}

hipError_t launch_best4_cross(const UpdArgs& a, const B4Args& b, hipStream_t s) {
  const int tiles_n = (a.t + 31) / 32;
  if (a.data_f64)
    hipLaunchKernelGGL(best4_cross_kernel<double>, dim3(tiles_n * tiles_n, a.gslabs), dim3(256), 0, s, a, b);
  else
    hipLaunchKernelGGL(best4_cross_kernel<float>, dim3(tiles_n * tiles_n, a.gslabs), dim3(256), 0, s, a, b);
  hipLaunchKernelGGL(best4_cross_reduce_kernel, dim3((a.t * a.t + 255) / 256), dim3(256), 0, s, a, b);
  return hipGetLastError();
}

// Keeps the update's record (the estimate of the candidate just evaluated).
__global__ void best4_keep_kernel(UpdArgs a, B4Args b, int q) {
  if (threadIdx.x == 0) b.recq[q] = a.recs[a.u];
}

// Cholesky factor of G over the occupied slots (compact order), one
// workgroup: right-looking, column by column.  A pivot that is not positive
// (a numerically dependent basis column) leaves a zero column: the solves
// below then give that unknown 0.
__global__ __launch_bounds__(1024) void best4_chol_kernel(UpdArgs a, B4Args b) {
  const int t = a.t, no = min(a.sc->n_occ, a.ell);
  const int* occ = a.sc->occ_slot;
  double* L = b.L;
  for (int idx = threadIdx.x; idx < no * no; idx += blockDim.x) {
    const int i = idx % no, j = idx / no;
    L[(int64_t)j * t + i] = (i >= j) ? a.G[(int64_t)occ[j] * t + occ[i]] : 0.0;
  }
  __syncthreads();
  __shared__ double piv;
  double gmax = 0.0;
  for (int i = 0; i < no; ++i) gmax = fmax(gmax, a.G[(int64_t)occ[i] * t + occ[i]]);
  const double tiny = (double)no * 2.220446049250313e-16 * gmax;
  for (int j = 0; j < no; ++j) {
    if (threadIdx.x == 0) {
      const double d = L[(int64_t)j * t + j];
      piv = d > tiny ? sqrt(d) : 0.0;
      L[(int64_t)j * t + j] = piv;
    }
    __syncthreads();
    const double p = piv;
    for (int i = j + 1 + threadIdx.x; i < no; i += blockDim.x)
      L[(int64_t)j * t + i] = p > 0.0 ? L[(int64_t)j * t + i] / p : 0.0;
    __syncthreads();
    // trailing update of the lower triangle, column by column
    const int rem = no - j - 1;
    for (int idx = threadIdx.x; idx < rem * rem; idx += blockDim.x) {
      const int i = j + 1 + idx % rem, c = j + 1 + idx / rem;
      if (i >= c) L[(int64_t)c * t + i] -= L[(int64_t)j * t + i] * L[(int64_t)j * t + c];
    }
    __syncthreads();
  }
}

// Right-hand sides, compact rows: which 0 -> M5 (no x l, Mm layout) holds
// S_J^T / l; which 1 -> T (no x no_prev) holds A_J^T A_{J_prev} assembled from
// the current Gram (unchanged previous columns), the previous Gram (kept x
// pruned) and the new-by-pruned products.
__global__ __launch_bounds__(256) void best4_rhs_kernel(UpdArgs a, B4Args b, int which) {
  __shared__ int occp[kMaxT];
  __shared__ int nop;
  const int t = a.t, n = a.ell, no = min(a.sc->n_occ, n);
  const int* occ = a.sc->occ_slot;
  if (which == 0) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)no * n) return;
    const int i = (int)(idx % no), r = (int)(idx / no);
    b.M5[(int64_t)r * t + i] = a.S[a.J[occ[i]] * n + r] / (double)n;
    return;
  }
  if (threadIdx.x == 0) {
    int c = 0;
    for (int j = 0; j < t; ++j)
      if (b.J_prev[j] >= 0) occp[c++] = j;
    nop = c;
  }
  __syncthreads();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)no * nop) return;
  const int i = (int)(idx % no), c = (int)(idx / no);
  const int si = occ[i], sj = occp[c];
  const bool j_kept = a.J[sj] == b.J_prev[sj];
  const bool i_kept = a.J[si] == b.J_prev[si];
  double v;
  if (j_kept) v = a.G[(int64_t)sj * t + si];
  else if (i_kept) v = b.G_prev[(int64_t)sj * t + si];
  else v = b.Xc[(int64_t)sj * t + si];
  b.T[(int64_t)c * t + i] = v;
}

// X = L^{-T} L^{-1} X in place, one thread per right-hand side (column c of
// no entries at c * t).  which 0: the l columns of M5; 1: the no_prev columns
// of T.
__global__ __launch_bounds__(64) void best4_solve_kernel(UpdArgs a, B4Args b, int which) {
  const int t = a.t, no = min(a.sc->n_occ, a.ell);
  int ncols;
  if (which == 0) {
    ncols = a.ell;
  } else {
    ncols = 0;
    for (int j = 0; j < t; ++j) ncols += b.J_prev[j] >= 0;
  }
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  double* x = (which == 0 ? b.M5 : b.T) + (int64_t)c * t;
  const double* L = b.L;
  for (int i = 0; i < no; ++i) {
    double v = x[i];
    for (int k = 0; k < i; ++k) v -= L[(int64_t)k * t + i] * x[k];
    const double d = L[(int64_t)i * t + i];
    x[i] = d > 0.0 ? v / d : 0.0;
  }
  for (int i = no - 1; i >= 0; --i) {
    double v = x[i];
    for (int k = i + 1; k < no; ++k) v -= L[(int64_t)i * t + k] * x[k];
    const double d = L[(int64_t)i * t + i];
    x[i] = d > 0.0 ? v / d : 0.0;
  }
}

// The selection state restricted to the new slots (the Alg. 4 factorisation
// of S over them gives their part of the residual fit of Alg. 6).
__global__ void best4_sc6_kernel(UpdArgs a, B4Args b) {
  constexpr int nw = (int)(sizeof(DevScalars) / sizeof(int32_t));
  for (int k = threadIdx.x; k < nw; k += blockDim.x)
    reinterpret_cast<int32_t*>(b.sc6)[k] = reinterpret_cast<const int32_t*>(a.sc)[k];
  __syncthreads();
  if (threadIdx.x == 0) b.sc6->n_occ = a.sc->n_new;
  for (int i = threadIdx.x; i < a.sc->n_new; i += blockDim.x) b.sc6->occ_slot[i] = a.sc->new_slot[i];
}

// r_A = S - S_J Pz over the columns the previous P covers (Pz: the rows of
// the slots that kept their column).
__global__ __launch_bounds__(256) void best4_ra_kernel(UpdArgs a, B4Args b) {
  __shared__ double red[4 * 16 * 64];
  const int n = a.ell, t = a.t;
  const int64_t np = b.n_prev;
  const int nmt = (n + 31) / 32;
  const int m0 = 32 * (blockIdx.x % nmt), n0 = 32 * (blockIdx.x / nmt);
  if (n0 >= np) return;
  double out[2][2][4];
  gemm32_f64(m0, n0, t,
             [&](int r, int k) {
               return (r < n && k < t && a.J[k] >= 0 && a.J[k] == b.J_prev[k]) ? a.S[a.J[k] * n + r] : 0.0;
             },
             [&](int k, int c) { return (k < t && c < np) ? b.Pprev[(int64_t)c * t + k] : 0.0; }, out, red);
  if ((threadIdx.x >> 6) == 0) {
    const int lane = threadIdx.x & 63, i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = m0 + 16 * x + k4 + 4 * v, c = n0 + 16 * y + i16;
          if (r < n && c < np) b.rA[(int64_t)c * n + r] = a.S[(int64_t)c * n + r] - out[x][y][v];
        }
  }
}

// P6 = Pz + D6 over the columns the previous P covers, P4 after them.
__global__ __launch_bounds__(256) void best4_p6_kernel(UpdArgs a, B4Args b) {
  const int t = a.t;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)t * a.n_obs) return;
  const int i = (int)(idx % t);
  const int64_t c = idx / t;
  const double* P4 = b.Pc;
  double* P6 = b.Pc + 2 * (int64_t)t * b.n_max;
  if (c < b.n_prev) {
    const bool kept = a.J[i] >= 0 && a.J[i] == b.J_prev[i];
    P6[idx] = (kept ? b.Pprev[idx] : 0.0) + b.D6[idx];
  } else {
    P6[idx] = P4[idx];
  }
}

// P7 = T P_prev over the columns the previous P covers (rows of the occupied
// slots; zero rows for empty slots), P4 after them.
__global__ __launch_bounds__(256) void best4_p7_kernel(UpdArgs a, B4Args b) {
  __shared__ double red[4 * 16 * 64];
  __shared__ int occp[kMaxT];
  __shared__ int nop;
  const int t = a.t, no = min(a.sc->n_occ, a.ell);
  const int64_t np = b.n_prev, nobs = a.n_obs;
  const double* P4 = b.Pc;
  double* P7 = b.Pc + 3 * (int64_t)t * b.n_max;
  const int nmt = (t + 31) / 32;
  const int m0 = 32 * (blockIdx.x % nmt), n0 = 32 * (blockIdx.x / nmt);
  if (n0 >= nobs) return;
  // columns after the previous P: P4's (slots m0 .. m0 + 31 of this tile)
  for (int idx = threadIdx.x; idx < 32 * 32; idx += blockDim.x) {
    const int i = m0 + idx % 32;
    const int64_t c = n0 + idx / 32;
    if (i < t && c >= np && c < nobs) P7[c * t + i] = P4[c * t + i];
  }
  if (n0 >= np) return;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int j = 0; j < t; ++j)
      if (b.J_prev[j] >= 0) occp[c++] = j;
    nop = c;
  }
  __syncthreads();
  const int kp = nop;
  // rows of empty slots are zero (this block's columns before np)
  if (m0 == 0) {
    for (int idx = threadIdx.x; idx < 32 * t; idx += blockDim.x) {
      const int i = idx % t;
      const int64_t c = n0 + idx / t;
      if (a.J[i] < 0 && c < np) P7[c * t + i] = 0.0;
    }
  }
  if (m0 >= no) return;
  double out[2][2][4];
  gemm32_f64(m0, n0, kp, [&](int i, int k) { return (i < no && k < kp) ? b.T[(int64_t)k * t + i] : 0.0; },
             [&](int k, int c) { return (k < kp && c < np) ? b.Pprev[(int64_t)c * t + occp[k]] : 0.0; }, out, red);
  if ((threadIdx.x >> 6) == 0) {
    const int lane = threadIdx.x & 63, i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = m0 + 16 * x + k4 + 4 * v;
          const int64_t c = n0 + 16 * y + i16;
          if (i < no && c < np) P7[c * t + a.sc->occ_slot[i]] = out[x][y][v];
        }
  }
}

// The smallest estimate wins (ties: the lowest q): its record becomes the
// update's, and the choice is kept.
__global__ void best4_choose_kernel(UpdArgs a, B4Args b) {
  if (threadIdx.x != 0) return;
  int best = 0;
  for (int q = 1; q < 4; ++q)
    if (b.recq[q].E2 < b.recq[best].E2) best = q;
  a.recs[a.u] = b.recq[best];
  *b.qstar = 4 + best;
}

// P = P_{q*} into the stream's P and the next update's P_prev.
__global__ __launch_bounds__(256) void best4_copy_kernel(UpdArgs a, B4Args b) {
  const int64_t n = (int64_t)a.t * a.n_obs;
  const double* src = b.Pc + (int64_t)(*b.qstar - 4) * a.t * b.n_max;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = src[i];
    b.Pout[i] = v;
    b.Pprev[i] = v;
  }
}

namespace {

// The Alg. 4 factorisation (Householder QR of S over the slots in a.sc, the
// thin Q, M = R'^{-1} Q^T), for t <= kAlg4Gemm.
void best4_factor(const UpdArgs& a, hipStream_t s) {
  const int E = (a.ell + 63) / 64;
  if (E <= 1 && a.t <= 16)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<1, 2, 8>), dim3(1), dim3(512), 0, s, a);
  else if (E <= 2 && a.t <= 64)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<2, 8, 8>), dim3(1), dim3(512), 0, s, a);
  else if (E <= 4 && a.t <= 112)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<4, 14, 8>), dim3(1), dim3(512), 0, s, a);
  else if (E <= 5 && a.t <= 152)
    hipLaunchKernelGGL((alg4_qr_reg_kernel<5, 19, 8>), dim3(1), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL(alg4_qr_kernel, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(alg4_q_kernel, dim3(a.t), dim3(64), 0, s, a);
  hipLaunchKernelGGL(alg4_m_kernel, dim3((a.ell + 3) / 4), dim3(256), alg4_m_lds(a.t), s, a);
}

// NA-Hutch++ (Alg. 8) of the coefficients in a.P, into a.recs[a.u].
void best4_hutch(const UpdArgs& a, hipStream_t s) {
  const int tiles = ((a.ell + 31) / 32) * ((a.t + 31) / 32) + ((a.t + 31) / 32) * ((a.t + 31) / 32);
  hipLaunchKernelGGL(hutch_gemm_kernel, dim3(tiles), dim3(256), 0, s, a);
  const int n3 = a.ell - a.n1 - a.n2;
  const int64_t s0 = (int64_t)a.ell * a.t;
  const int64_t s1 = (int64_t)a.n1 * a.n2 + (int64_t)a.n1 * a.t + (int64_t)a.n1 * n3 + (int64_t)n3 * a.n2;
  const int64_t s2 = (int64_t)a.n1 * a.n2;
  hipLaunchKernelGGL(hutch_mid_kernel, dim3((unsigned)((s0 + 255) / 256)), dim3(256), 0, s, a, 0);
  hipLaunchKernelGGL(hutch_mid_kernel, dim3((unsigned)((s1 + 255) / 256)), dim3(256), 0, s, a, 1);
  hipLaunchKernelGGL(hutch_mid_kernel, dim3((unsigned)((s2 + 255) / 256)), dim3(256), 0, s, a, 2);
  const int E = (a.n2 + 63) / 64, nv = 3 * a.n1;
  if (a.n1 > 0 && E <= 1 && nv <= 8 * 4)
    hipLaunchKernelGGL((hutch_small_reg_kernel<1, 4, 8>), dim3(1), dim3(512), 0, s, a);
  else if (a.n1 > 0 && E <= 2 && nv <= 8 * 19)
    hipLaunchKernelGGL((hutch_small_reg_kernel<2, 19, 8>), dim3(1), dim3(512), 0, s, a);
  else if (a.n1 > 0 && E <= 3 && nv <= 8 * 29)
    hipLaunchKernelGGL((hutch_small_reg_kernel<3, 29, 8>), dim3(1), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL(hutch_small_kernel, dim3(1), dim3(1024), 0, s, a);
}

}  // namespace

hipError_t launch_best4(const UpdArgs& a, const B4Args& b, hipStream_t s) {
  alg4_m_attributes();
  const int t = a.t, n = a.ell;
  const int64_t tn = (int64_t)t * b.n_max;
  const unsigned pcols = (unsigned)(((t + 31) / 32) * ((a.n_obs + 31) / 32));
  hipLaunchKernelGGL(best4_keep_kernel, dim3(1), dim3(64), 0, s, a, b, 0);
  // Alg. 5
  hipLaunchKernelGGL(best4_chol_kernel, dim3(1), dim3(1024), 0, s, a, b);
  hipLaunchKernelGGL(best4_rhs_kernel, dim3((unsigned)(((int64_t)t * n + 255) / 256)), dim3(256), 0, s, a, b, 0);
  hipLaunchKernelGGL(best4_solve_kernel, dim3((n + 63) / 64), dim3(64), 0, s, a, b, 0);
  UpdArgs a5 = a;
  a5.Mm = b.M5;
  a5.P = b.Pc + tn;
  hipLaunchKernelGGL(alg4_pgemm_kernel, dim3(pcols), dim3(256), 0, s, a5);
  // Alg. 6 (over the previous columns; the rest are P4's)
  if (b.n_prev > 0) {
    hipLaunchKernelGGL(best4_sc6_kernel, dim3(1), dim3(256), 0, s, a, b);
    UpdArgs a6 = a;
    a6.sc = b.sc6;
    a6.QR = b.QR6;
    a6.qr_tau = b.tau6;
    a6.Qm = b.Qm6;
    a6.Mm = b.Mm6;
    a6.recs = b.scratch_rec;
    a6.u = 0;
    best4_factor(a6, s);
    hipLaunchKernelGGL(best4_ra_kernel, dim3((unsigned)(((n + 31) / 32) * ((b.n_prev + 31) / 32))), dim3(256), 0,
                       s, a, b);
    a6.S = b.rA;
    a6.n_obs = b.n_prev;
    a6.P = b.D6;
    hipLaunchKernelGGL(alg4_pgemm_kernel, dim3((unsigned)(((t + 31) / 32) * ((b.n_prev + 31) / 32))), dim3(256),
                       0, s, a6);
  }
  hipLaunchKernelGGL(best4_p6_kernel, dim3((unsigned)(((int64_t)t * a.n_obs + 255) / 256)), dim3(256), 0, s, a,
                     b);
  // Alg. 7
  if (b.n_prev > 0) {
    hipLaunchKernelGGL(best4_rhs_kernel, dim3((unsigned)(((int64_t)t * t + 255) / 256)), dim3(256), 0, s, a, b, 1);
    hipLaunchKernelGGL(best4_solve_kernel, dim3((t + 63) / 64), dim3(64), 0, s, a, b, 1);
  }
  hipLaunchKernelGGL(best4_p7_kernel, dim3(pcols), dim3(256), 0, s, a, b);
  // estimates of Algs. 5, 6, 7 and the choice
  for (int q = 1; q < 4; ++q) {
    UpdArgs aq = a;
    aq.P = b.Pc + q * tn;
    best4_hutch(aq, s);
    hipLaunchKernelGGL(best4_keep_kernel, dim3(1), dim3(64), 0, s, a, b, q);
  }
  hipLaunchKernelGGL(best4_choose_kernel, dim3(1), dim3(64), 0, s, a, b);
  const int64_t nel = (int64_t)t * a.n_obs;
  hipLaunchKernelGGL(best4_copy_kernel, dim3((unsigned)std::min<int64_t>(1024, (nel + 255) / 256)), dim3(256), 0,
                     s, a, b);
  return hipGetLastError();
}

size_t hutch_work_doubles(int ell, int t) {
  return (size_t)hutch_work_quarter(ell) * 5 + (size_t)ell * t * 2;
}

}  // namespace rid
