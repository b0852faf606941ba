// One-shot sketch of a block of columns (eq. random_sketch; the column norms
// of Alg. 3 step 13) with no stream state: S = Omega A and ||a_j||^2 for b
// device columns, with the same sketch and reduction kernels the streams use.
//
// Work space per call: the device table of column addresses, the per-slab
// partial sketches [slab][b][l_pad] and partial norms [slab][b], and a
// non-finite flag.  The slab geometry depends only on (form, l, m, b): the
// slab count a stream would use for a lookahead batch of b columns, lowered
// where the partials would pass kOneShotMaxBytes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "rid_internal.h"

using namespace rid;

namespace {

// Largest work space of one call (either entry point).
constexpr size_t kOneShotMaxBytes = size_t(128) << 20;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct OneShot {
  SketchArgs a;
  size_t off_flag, off_norm, off_part, bytes;
};

// Column table, flag zeroed (the reduction only ever sets it).
__global__ void oneshot_setup_kernel(uint64_t* table, uint64_t base, uint64_t stride, int32_t b,
                                     int32_t* flag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < b) table[j] = base + (uint64_t)j * stride;
  if (j == 0) *flag = 0;
}

rid_status oneshot_plan(int32_t prec, uint64_t seed, int32_t ell, int64_t m, const void* d_cols, int64_t ld,
                        int32_t b, double* d_S, double* d_colsq, OneShot* p, std::string* err) {
  if (prec < RID_SKETCH_F64 || prec > RID_SKETCH_FP8) {
    *err = "unknown sketch precision";
    return RID_EINVAL;
  }
  if (ell < 1 || ell > kMaxEll || m < 1 || b < 1 || ld < m || !d_cols || !d_S || !d_colsq) {
    *err = "bad sizes or null pointers (need 1 <= ell <= 512, m >= 1, b >= 1, ld >= m)";
    return RID_EINVAL;
  }
  const int64_t es = prec == RID_SKETCH_F64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(d_cols) % 16 != 0 || (ld * es) % 16 != 0) {
    *err = "columns must start on 16-byte boundaries (pointer and ld * element size)";
    return RID_EINVAL;
  }
  SketchArgs& a = p->a;
  a = SketchArgs{};
  sketch_tile_geometry(prec, ell, 0, &a.ell_pad, &a.n_mt, &a.rbw);
  a.wide = 0;
  const int cpw = sketch_cols_per_wg(prec, 0);
  a.n_nt = (b + cpw - 1) / cpw;
  a.c0 = 0;
  a.b = b;
  a.b_max = b;
  a.m = m;
  a.ell = ell;
  a.seed = seed;
  const size_t psize = prec == RID_SKETCH_F64 ? 8 : 4;
  const size_t fixed = align256((size_t)b * 8) + 256;
  const size_t per_slab = (size_t)b * a.ell_pad * psize + (size_t)b * 8;
  // the slab count of a stream's lookahead batch of b columns ...
  const int64_t target = std::max<int64_t>(1, 2048 / (a.n_mt * a.n_nt));
  int64_t rows = (m + target - 1) / target;
  // ... and no more slabs than the work space holds
  const int64_t fit = (int64_t)((kOneShotMaxBytes - fixed - 512) / per_slab);
  if (fit < 1) {
    *err = "b x l too large for the one-shot work space";
    return RID_ECAPACITY;
  }
  rows = std::max<int64_t>(rows, (m + fit - 1) / fit);
  rows = (rows + 255) / 256 * 256;
  rows = std::max<int64_t>(rows, 256);
  if (rows > sketch_slab_cap(prec)) {
    *err = "the partial sketches of " + std::to_string(b) + " columns of " + std::to_string(m) +
           " rows pass the " + std::to_string(kOneShotMaxBytes >> 20) + " MiB work space; push fewer columns";
    return RID_ECAPACITY;
  }
  a.slab_rows = rows;
  a.n_slabs = (int)((m + rows - 1) / rows);
  p->off_flag = align256((size_t)b * 8);
  p->off_norm = p->off_flag + 256;
  p->off_part = p->off_norm + align256((size_t)a.n_slabs * b * 8);
  p->bytes = p->off_part + align256((size_t)a.n_slabs * b * a.ell_pad * psize);
  a.S = d_S;
  a.colsq = d_colsq;
  return RID_OK;
}

// Enqueues the sketch of the planned call with its work space at `ws`.
hipError_t oneshot_launch(int32_t prec, OneShot& p, char* ws, const void* d_cols, int64_t ld,
                          int32_t* d_nonfinite, hipStream_t s) {
  SketchArgs& a = p.a;
  const int64_t es = prec == RID_SKETCH_F64 ? 8 : 4;
  a.colptr = reinterpret_cast<const uint64_t*>(ws);
  a.nonfinite = d_nonfinite ? d_nonfinite : reinterpret_cast<int32_t*>(ws + p.off_flag);
  a.normpart = reinterpret_cast<double*>(ws + p.off_norm);
  a.part = ws + p.off_part;
  hipLaunchKernelGGL(oneshot_setup_kernel, dim3((a.b + 255) / 256), dim3(256), 0, s,
                     reinterpret_cast<uint64_t*>(ws), (uint64_t)reinterpret_cast<uintptr_t>(d_cols),
                     (uint64_t)(ld * es), a.b, a.nonfinite);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_sketch(prec, a, s)) != hipSuccess) return e;
  return launch_sketch_reduce(prec, a, s);
}

// Work space of rid_sketch_columns_noalloc: one array per device (each GPU the
// library runs on holds it until the process ends), as large as the largest
// work space of one call.  In host code the name stands for a host-side
// symbol, not the device address: kernels get the address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) char scratch[kOneShotMaxBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
rid_status scratch_address(void** out, std::string* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    *err = "no usable HIP device";
    return RID_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      *err = std::string("hipGetSymbolAddress of the work space: ") + hipGetErrorString(e);
      return RID_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RID_OK;
}

}  // namespace

extern "C" {

rid_status rid_sketch_columns_noalloc(int32_t sketch_prec, uint64_t omega_seed, int32_t ell, int64_t m,
                                      const void* d_cols, int64_t ld, int32_t b, double* d_S, double* d_colsq,
                                      int32_t* d_nonfinite, void* stream) {
  OneShot p;
  std::string err;
  rid_status st = oneshot_plan(sketch_prec, omega_seed, ell, m, d_cols, ld, b, d_S, d_colsq, &p, &err);
  if (st != RID_OK) return rid_set_global_error(st, "rid_sketch_columns_noalloc: " + err);
  if (p.bytes > kOneShotMaxBytes)
    return rid_set_global_error(RID_ECAPACITY, "rid_sketch_columns_noalloc: needs " + std::to_string(p.bytes) +
                                                   " bytes of work space, the maximum is " +
                                                   std::to_string(kOneShotMaxBytes));
  void* ws = nullptr;
  if ((st = scratch_address(&ws, &err)) != RID_OK)
    return rid_set_global_error(st, "rid_sketch_columns_noalloc: " + err);
  const hipError_t e = oneshot_launch(sketch_prec, p, reinterpret_cast<char*>(ws), d_cols, ld, d_nonfinite,
                                      reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return rid_set_global_error(RID_EDEVICE, std::string("rid_sketch_columns_noalloc: ") + hipGetErrorString(e));
  return RID_OK;
}

rid_status rid_sketch_columns(int32_t sketch_prec, uint64_t omega_seed, int32_t ell, int64_t m,
                              const void* d_cols, int64_t ld, int32_t b, double* d_S, double* d_colsq,
                              int32_t* d_nonfinite, void* stream) {
  OneShot p;
  std::string err;
  rid_status st = oneshot_plan(sketch_prec, omega_seed, ell, m, d_cols, ld, b, d_S, d_colsq, &p, &err);
  if (st != RID_OK) return rid_set_global_error(st, "rid_sketch_columns: " + err);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, p.bytes, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return rid_set_global_error(RID_ENOMEM, "rid_sketch_columns: hipMallocAsync of " + std::to_string(p.bytes) +
                                                " bytes: " + hipGetErrorString(e));
  }
  e = oneshot_launch(sketch_prec, p, reinterpret_cast<char*>(ws), d_cols, ld, d_nonfinite, s);
  const hipError_t e2 = hipFreeAsync(ws, s);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess)
    return rid_set_global_error(RID_EDEVICE, std::string("rid_sketch_columns: ") + hipGetErrorString(e));
  return RID_OK;
}

}  // extern "C"
