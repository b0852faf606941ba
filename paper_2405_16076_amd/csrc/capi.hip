// Host runtime and C ABI of the streaming randomized ID (include/rid.h).
//
// A handle owns the device state of one stream.  Pushed columns are recorded
// in a column-pointer table (BORROW: the caller's addresses; COPY: slots of a
// device ring the columns are copied into).  Sketches are launched over up to
// `lookahead` buffered columns at a time (the sketch of a column does not
// depend on its batch), and the update of Alg. 3 is enqueued for every group
// of t consecutive sketched columns.  No device-to-host traffic happens except
// in the getters.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <memory>
#include <vector>

#include "rid_internal.h"

namespace rid {

// ---------------------------------------------------------------------------
// reconstruct: out(:, jj) = sum over occupied slots i of C(:, i) P(i, j0 + jj)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void reconstruct_kernel(const T* __restrict__ C, int64_t ldc,
                                                          const double* __restrict__ P, int t,
                                                          const int64_t* __restrict__ J, int64_t m,
                                                          int64_t j0, int c, T* out, int64_t ld) {
  constexpr int CB = 16;
  __shared__ double pt[kMaxT][CB];
  __shared__ int occ[kMaxT];
  __shared__ int nocc;
  const int tid = threadIdx.x;
  const int cb0 = blockIdx.y * CB;
  if (tid == 0) {
    int no = 0;
    for (int i = 0; i < t; ++i)
      if (J[i] >= 0) occ[no++] = i;
    nocc = no;
  }
  for (int idx = tid; idx < t * CB; idx += blockDim.x) {
    const int i = idx / CB, jj = idx % CB;
    pt[i][jj] = (cb0 + jj < c) ? P[(j0 + cb0 + jj) * t + i] : 0.0;
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + tid;
  if (row >= m) return;
  double acc[CB];
#pragma unroll
  for (int jj = 0; jj < CB; ++jj) acc[jj] = 0.0;
  for (int q = 0; q < nocc; ++q) {
    const int i = occ[q];
    const double x = (double)C[(int64_t)i * ldc + row];
#pragma unroll
    for (int jj = 0; jj < CB; ++jj) acc[jj] = fma(x, pt[i][jj], acc[jj]);
  }
#pragma unroll
  for (int jj = 0; jj < CB; ++jj)
    if (cb0 + jj < c) out[(int64_t)(cb0 + jj) * ld + row] = (T)acc[jj];
}

__global__ void init_state_kernel(int64_t* J, double* tau_old, int t, DevScalars* sc, uint64_t* slot_ptr,
                                  const char* pool, int64_t col_bytes) {
  const int i = threadIdx.x;
  if (i < t) {
    J[i] = -1;
    tau_old[i] = 1.0;
    slot_ptr[i] = reinterpret_cast<uint64_t>(pool + (int64_t)i * col_bytes);
  }
  if (i == 0) {
    sc->nonfinite = 0;
    sc->n_new = 0;
    sc->n_occ = 0;
    sc->rank = 0;
  }
}

}  // namespace rid

using namespace rid;

struct rid_batch;

struct rid_stream {
  rid_config cfg;
  hipStream_t s = nullptr;
  int dev = 0;
  int ell = 0, k = 0, t = 0, n1 = 0, n2 = 0, prec = 0, esize = 4, data_f64 = 0;
  int64_t m = 0, n_max = 0;
  double fill_mult = 0.0;
  // sketch geometry
  int ell_pad = 0, n_mt = 0, rbw = 0, wide = 0, cols_per_wg = 0, b_max = 0, n_slabs = 0;
  int64_t slab_rows = 0;
  int gslabs = 0;
  int64_t gslab_rows = 0;
  int64_t ldc = 0;
  // device memory
  std::vector<void*> allocs;
  std::vector<size_t> alloc_bytes;
  size_t dev_bytes = 0;
  double *S = nullptr, *colsq = nullptr, *W = nullptr, *hv = nullptr, *Qs = nullptr, *Ys = nullptr;
  double* SST[2] = {nullptr, nullptr};  // SS^T after the last enqueued update (ping-pong)
  int sst_cur = 0;
  int nzmax = 0;                        // updates per batch (slots of W and hv)
  double* Fu = nullptr;
  double* Tu = nullptr;   // tr(SS^T) per update
  int32_t* skipu = nullptr;
  double *tauC = nullptr, *tauD = nullptr, *tau_old = nullptr, *tauC_hist = nullptr,
         *tauD_hist = nullptr;
  double *G = nullptr, *gpart = nullptr, *QR = nullptr, *qr_tau = nullptr, *P = nullptr;
  double *Qm = nullptr, *Mm = nullptr;
  double *Y = nullptr, *PPt = nullptr, *hw = nullptr;
  int64_t *J = nullptr, *J_hist = nullptr;
  uint64_t* colptr_dev = nullptr;
  uint64_t* colptr_host = nullptr;  // pinned
  hipEvent_t colptr_ev = nullptr;   // after the last upload of colptr_host
  bool colptr_pending = false;
  void* cpool = nullptr;
  uint64_t* slot_ptr = nullptr;  // t column addresses (split Gram: pool or this flush's snapshots)
  void* ring = nullptr;
  int64_t ring_cap = 0, ring_ld = 0;
  void* part = nullptr;
  double* normpart = nullptr;
  DevScalars* sc = nullptr;
  rid_update* recs = nullptr;
  int64_t max_updates = 0;
  // host counters
  int64_t n_pushed = 0, n_sketched = 0, n_uploaded = 0, n_updates = 0, last_nobs = 0;
  bool finalized = false, failed = false;
  rid_status last_status = RID_OK;
  std::string last_err;
  // live timing: event pairs recorded on the stream around launch groups
  struct Mark {
    hipEvent_t a, b;
    int kind;        // 0 sketch, 1 reduce, 2 update, 3 gram, 4 coefficient phases (second stream)
    double bytes;
    hipStream_t on;  // stream the events are recorded on
    int64_t aux;     // gram: the flush's first column at its last update (split Gram), -2 for a
                     // run of updates' Grams in one pass (bytes: its reads), else -1
    int nu = 1;      // updates of a run
  };
  bool profiling = false;
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  // member of a batch: pushes go through the batch; results reach the
  // caller's stream `join` through `join_ev`
  rid_batch* owner = nullptr;
  hipStream_t join = nullptr;
  hipEvent_t join_ev = nullptr;
  // Alg. 4 and Alg. 8 of update u run on `side` against snapshots of the
  // selection state (sc_hist[u], Ghist[u], J_hist[u]) while `s` goes on with
  // the selection of update u + 1; side_ev marks the newest side work.
  hipStream_t side = nullptr;
  hipEvent_t side_ev = nullptr;
  bool side_used = false;
  DevScalars* sc_hist = nullptr;
  double* Ghist = nullptr;
  // The coefficient phases of the updates of one flush run on `side` as
  // batched launches, cgroup updates at a time, each with its own slice of
  // QR, qr_tau, Qm, Mm, Y, PPt and hw; P of every update but the last of the
  // flush goes to a slice of Pz.  Their argument tables go to ctab_dev from a
  // ring of pinned host slots.
  int cgroup = 1;
  // RID_COEFF_BEST4: the candidates, the kept P of the previous update and
  // the work space of Algs. 5-7 (B4Args); Xc has one t x t slot per update of
  // a flush, recq four records and qstar one choice per update
  bool best4 = false;
  bool gram_split = false;  // binary32 Gram on the bfloat16 matrix cores
  // Split Grams of runs of consecutive updates of a flush in one pass
  // (stand-alone streams in ALG4 mode): partials with leading dimension
  // gld = max(t, 256) and the running list
  bool gram_merge = false;
  int gld = 0;
  GramRun* grun = nullptr;
  double *b4_Pc = nullptr, *b4_Pprev = nullptr, *b4_M5 = nullptr, *b4_L = nullptr, *b4_T = nullptr;
  double *b4_rA = nullptr, *b4_D6 = nullptr, *b4_QR6 = nullptr, *b4_tau6 = nullptr, *b4_Qm6 = nullptr;
  double *b4_Mm6 = nullptr, *b4_Xc = nullptr;
  DevScalars* b4_sc6 = nullptr;
  rid_update *b4_rec = nullptr, *b4_recq = nullptr;
  int32_t* b4_qstar = nullptr;
  double* Pz = nullptr;
  double* SSTk = nullptr;   // nzmax slots of l x l: each update's SS^T (sst_keep)
  // the next flush's SS^T batch rewrites SSTk: it waits for the side stream's
  // coefficient phases of the previous flush (coeff_ev)
  hipEvent_t coeff_ev = nullptr;
  bool coeff_pending = false;
  // after a reset that left them running: the next sketch reduction, which
  // rewrites S from column 0, waits for them first
  bool reduce_wait = false;
  static constexpr int kTabSlots = 3;
  char* ctab_host[kTabSlots] = {nullptr, nullptr, nullptr};
  hipEvent_t ctab_ev[kTabSlots] = {nullptr, nullptr, nullptr};
  bool ctab_used[kTabSlots] = {false, false, false};
  int ctab_slot = 0;
  char* ctab_dev = nullptr;
  size_t ctab_cap = 0;
};

static thread_local std::string g_last_err;


// Status of a call that has no handle (its message is read with
// rid_last_error(NULL, ...)).
rid_status rid::rid_set_global_error(rid_status st, const std::string& msg) {
  g_last_err = msg;
  return st;
}

static rid_status fail(rid_stream* h, rid_status st, const std::string& msg) {
  if (h) {
    h->last_err = msg;
    if (st == RID_EDEVICE || st == RID_ENUMERIC) {
      h->failed = true;
      h->last_status = st;
    }
  } else {
    g_last_err = msg;
  }
  return st;
}

#define RID_HIP(h, expr)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((h), RID_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static rid_status dalloc(rid_stream* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(h, RID_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  h->allocs.push_back(*p);
  h->alloc_bytes.push_back(bytes);
  h->dev_bytes += bytes;
  return RID_OK;
}

template <typename T>
static rid_status dalloc_t(rid_stream* h, T** p, size_t count) {
  void* v = nullptr;
  rid_status st = dalloc(h, &v, count * sizeof(T));
  *p = reinterpret_cast<T*>(v);
  return st;
}

static void dfree(rid_stream* h, void* p) {
  for (size_t i = 0; i < h->allocs.size(); ++i)
    if (h->allocs[i] == p) {
      (void)hipFree(p);
      h->dev_bytes -= h->alloc_bytes[i];
      h->allocs.erase(h->allocs.begin() + (long)i);
      h->alloc_bytes.erase(h->alloc_bytes.begin() + (long)i);
      return;
    }
}

static void free_all(rid_stream* h) {
  for (auto& mk : h->marks) {
    (void)hipEventDestroy(mk.a);
    (void)hipEventDestroy(mk.b);
  }
  h->marks.clear();
  for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
  h->event_pool.clear();
  if (h->side) (void)hipStreamSynchronize(h->side);
  for (int i = 0; i < rid_stream::kTabSlots; ++i) {
    if (h->ctab_host[i]) (void)hipHostFree(h->ctab_host[i]);
    if (h->ctab_ev[i]) (void)hipEventDestroy(h->ctab_ev[i]);
    h->ctab_host[i] = nullptr;
    h->ctab_ev[i] = nullptr;
  }
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  h->alloc_bytes.clear();
  if (h->colptr_host) (void)hipHostFree(h->colptr_host);
  h->colptr_host = nullptr;
  if (h->side) (void)hipStreamSynchronize(h->side);
  if (h->side_ev) (void)hipEventDestroy(h->side_ev);
  if (h->coeff_ev) (void)hipEventDestroy(h->coeff_ev);
  h->coeff_ev = nullptr;
  if (h->colptr_ev) (void)hipEventDestroy(h->colptr_ev);
  h->colptr_ev = nullptr;
  if (h->side) (void)hipStreamDestroy(h->side);
  h->side_ev = nullptr;
  h->side = nullptr;
}

static bool wide_applies(const rid_stream* h) {
  return h->prec == RID_SKETCH_BF16 && h->ell > 128 && h->ell <= 320;
}

// Work split of the sketch.  Both bf16 splits give the same l_pad, so the
// partial buffers fit either.
static void set_tile(rid_stream* h, bool wide) {
  h->wide = (wide && wide_applies(h)) ? 1 : 0;
  sketch_tile_geometry(h->prec, h->ell, h->wide, &h->ell_pad, &h->n_mt, &h->rbw);
  h->cols_per_wg = sketch_cols_per_wg(h->prec, h->wide);
}

static int auto_lookahead(const rid_config* c) {
  int la = c->lookahead > 0 ? c->lookahead : 1024;
  la = std::max(la, 2 * c->t);
  return (int)std::min<int64_t>(la, std::max<int64_t>(c->n_max, 1));
}

extern "C" {

rid_status rid_config_default(rid_config* cfg) {
  if (!cfg) return RID_EINVAL;
  memset(cfg, 0, sizeof(*cfg));
  cfg->data_dtype = RID_F32;
  cfg->sketch_prec = RID_SKETCH_F32;
  cfg->omega_seed = 1;
  cfg->select_seed = 2;
  cfg->delta = 0.05;
  cfg->eps = 0.5;
  cfg->c_sample = 1.0;
  cfg->ridge_floor = 1e-8;
  return RID_OK;
}

const char* rid_status_string(rid_status s) {
  switch (s) {
    case RID_OK: return "RID_OK";
    case RID_EINVAL: return "RID_EINVAL: invalid argument";
    case RID_ENOMEM: return "RID_ENOMEM: allocation failed";
    case RID_EDEVICE: return "RID_EDEVICE: HIP error";
    case RID_ESTATE: return "RID_ESTATE: call not valid in this state";
    case RID_ECAPACITY: return "RID_ECAPACITY: more than n_max columns";
    case RID_ENUMERIC: return "RID_ENUMERIC: non-finite input or numerical breakdown";
    case RID_ENOTSUP: return "RID_ENOTSUP: configuration not supported";
  }
  return "unknown rid_status";
}

rid_status rid_last_error(rid_stream* h, char* buf, size_t n) {
  if (!buf || n == 0) return RID_EINVAL;
  const std::string& m = h ? h->last_err : g_last_err;
  snprintf(buf, n, "%s", m.c_str());
  return RID_OK;
}

static rid_status validate(const rid_config* c) {
  if (c->m < 1) return fail(nullptr, RID_EINVAL, "m must be >= 1");
  if (c->ell < 4 || c->ell > kMaxEll) return fail(nullptr, RID_EINVAL, "ell must be in [4, 512]");
  if (c->k < 1 || c->k > c->ell) return fail(nullptr, RID_EINVAL, "k must be in [1, ell]");
  if (c->t < 1 || c->t > c->ell || c->t > kMaxT)
    return fail(nullptr, RID_EINVAL, "t must be in [1, min(ell, 256)]");
  if (c->n_max < 1) return fail(nullptr, RID_EINVAL, "n_max must be >= 1");
  if (c->data_dtype != RID_F32 && c->data_dtype != RID_F64)
    return fail(nullptr, RID_EINVAL, "unknown data dtype");
  if (c->sketch_prec < RID_SKETCH_F64 || c->sketch_prec > RID_SKETCH_FP8)
    return fail(nullptr, RID_EINVAL, "unknown sketch precision");
  if ((c->sketch_prec == RID_SKETCH_F64) != (c->data_dtype == RID_F64))
    return fail(nullptr, RID_EINVAL, "the f64 sketch needs f64 data and the others f32 data");
  if (!(c->delta > 0.0 && c->delta < 1.0) || !(c->eps > 0.0) || !(c->c_sample > 0.0) ||
      !(c->ridge_floor >= 0.0))
    return fail(nullptr, RID_EINVAL, "delta, eps, c_sample or ridge_floor out of range");
  const int n1 = c->hutch_n1 > 0 ? c->hutch_n1 : c->ell / 4;
  const int n2 = c->hutch_n2 > 0 ? c->hutch_n2 : c->ell / 2;
  if (n1 < 1 || n2 <= n1 || n1 + n2 >= c->ell)
    return fail(nullptr, RID_EINVAL, "need 1 <= n1 < n2 and n1 + n2 < ell");
  if (n1 > kMaxEll / 4) return fail(nullptr, RID_ENOTSUP, "n1 above 128 is not supported");
  if (c->lookahead < 0) return fail(nullptr, RID_EINVAL, "lookahead must be >= 0");
  if (c->sketch_tile < RID_TILE_AUTO || c->sketch_tile > RID_TILE_WIDE)
    return fail(nullptr, RID_EINVAL, "unknown sketch_tile");
  if (c->sketch_tile == RID_TILE_WIDE && !(c->sketch_prec == RID_SKETCH_BF16 && c->ell > 128 && c->ell <= 320))
    return fail(nullptr, RID_ENOTSUP, "the wide sketch tile needs the bf16 form and 128 < ell <= 320");
  if (c->coeff_mode != RID_COEFF_ALG4 && c->coeff_mode != RID_COEFF_BEST4)
    return fail(nullptr, RID_EINVAL, "unknown coeff_mode");
  if (c->coeff_mode == RID_COEFF_BEST4 && c->t > kAlg4Gemm)
    return fail(nullptr, RID_ENOTSUP, "RID_COEFF_BEST4 needs t <= 154");
  if (c->gram_mode < RID_GRAM_AUTO || c->gram_mode > RID_GRAM_SPLIT)
    return fail(nullptr, RID_EINVAL, "unknown gram_mode");
  if (c->gram_mode == RID_GRAM_SPLIT && c->data_dtype != RID_F32)
    return fail(nullptr, RID_EINVAL, "RID_GRAM_SPLIT needs RID_F32 data");
  if (c->gram_mode == RID_GRAM_SPLIT && c->coeff_mode == RID_COEFF_BEST4)
    return fail(nullptr, RID_ENOTSUP, "RID_COEFF_BEST4 needs binary64 Gram products (RID_GRAM_AUTO or EXACT)");
  return RID_OK;
}

static rid_status init_stream(const rid_config* cfg, void* stream, rid_stream** out, bool member);

rid_status rid_init_stream(const rid_config* cfg, void* stream, rid_stream** out) {
  return init_stream(cfg, stream, out, false);
}

}  // extern "C"

// A member of a batch runs its coefficient phases through the batch's own
// launches (no tables of its own); its slices of P are capped at 256 MiB.
static rid_status init_stream(const rid_config* cfg, void* stream, rid_stream** out, bool member) {
  if (!cfg || !out) return fail(nullptr, RID_EINVAL, "null argument");
  *out = nullptr;
  rid_status st = validate(cfg);
  if (st != RID_OK) return st;
  if (member && cfg->coeff_mode == RID_COEFF_BEST4)
    return fail(nullptr, RID_ENOTSUP, "RID_COEFF_BEST4 is not supported for batch members");
  rid_stream* h = new rid_stream();
  h->cfg = *cfg;
  h->s = reinterpret_cast<hipStream_t>(stream);
  if (hipGetDevice(&h->dev) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    return fail(nullptr, RID_EDEVICE, "no HIP device");
  }
  h->m = cfg->m;
  h->ell = cfg->ell;
  h->k = cfg->k;
  h->t = cfg->t;
  h->n1 = cfg->hutch_n1 > 0 ? cfg->hutch_n1 : cfg->ell / 4;
  h->n2 = cfg->hutch_n2 > 0 ? cfg->hutch_n2 : cfg->ell / 2;
  h->prec = cfg->sketch_prec;
  h->data_f64 = cfg->data_dtype == RID_F64;
  h->esize = h->data_f64 ? 8 : 4;
  h->n_max = cfg->n_max;
  {
    const double k = cfg->k;
    h->fill_mult = cfg->c_sample * (k * log(k) + k * log(1.0 / cfg->delta) / cfg->eps) / cfg->t;
  }
  // sketch geometry
  set_tile(h, cfg->sketch_tile == RID_TILE_WIDE);
  h->b_max = auto_lookahead(cfg);
  {
    const int n_nt = (h->b_max + h->cols_per_wg - 1) / h->cols_per_wg;
    const int64_t cap = sketch_slab_cap(h->prec);
    const int64_t target = std::max<int64_t>(1, 2048 / (h->n_mt * n_nt));
    int64_t rows = (h->m + target - 1) / target;
    rows = (rows + 255) / 256 * 256;
    rows = std::min(std::max<int64_t>(rows, 256), cap);
    h->slab_rows = rows;
    h->n_slabs = (int)((h->m + rows - 1) / rows);
  }
  {
    // Gram slabs: about two 1024-thread workgroups per compute unit
    const int tt = (h->t + 159) / 160;
    const int64_t target = std::max<int64_t>(1, 512 / (tt * tt));
    int64_t rows = (h->m + target - 1) / target;
    rows = (rows + 255) / 256 * 256;
    rows = std::max<int64_t>(rows, 1024);
    h->gslab_rows = rows;
    h->gslabs = (int)((h->m + rows - 1) / rows);
  }
  h->ldc = (h->m + 63) / 64 * 64;
  h->max_updates = (h->n_max + h->t - 1) / h->t + 1;
  h->nzmax = h->b_max / h->t + 2;
  {
    // updates per batched coefficient launch: all of a flush.  Above
    // kAlg4Gemm every update forms its own P (t x n_max), so the group stops
    // where those slices would pass 1 GiB (256 MiB for a batch member).
    h->cgroup = h->nzmax;
    if (h->t > kAlg4Gemm) {
      const double pbytes = (double)h->t * (double)h->n_max * 8.0;
      const int by_mem = (int)std::max(1.0, std::floor((member ? 268435456.0 : 1073741824.0) / pbytes));
      h->cgroup = std::min(h->nzmax, by_mem);
    }
  }
  h->best4 = cfg->coeff_mode == RID_COEFF_BEST4;
  h->gram_split = !h->data_f64 && (cfg->gram_mode == RID_GRAM_SPLIT ||
                                   (cfg->gram_mode == RID_GRAM_AUTO && !h->best4));
  if (h->best4) h->cgroup = 1;   // each update's choice feeds the next one's Algs. 6 and 7
  h->gram_merge = h->gram_split && !h->best4 && !member;
  h->gld = h->gram_merge ? std::max(h->t, kGramRunCols) : h->t;
  const size_t ell = h->ell, t = h->t, cg = h->cgroup;
  const size_t psize = (h->prec == RID_SKETCH_F64) ? 8 : 4;
#define ALLOC(ptr, n) \
  if ((st = dalloc_t(h, &(ptr), (n))) != RID_OK) goto fail_alloc;
  {
    ALLOC(h->S, ell * h->n_max);
    ALLOC(h->colsq, h->n_max);
    ALLOC(h->SST[0], ell * ell);
    ALLOC(h->SST[1], ell * ell);
    ALLOC(h->W, ell * ell * h->nzmax);
    ALLOC(h->hv, 6 * ell * h->nzmax);
    ALLOC(h->Qs, ell * ell * h->nzmax);
    ALLOC(h->Ys, ell * 2 * t * h->nzmax);
    ALLOC(h->Fu, (size_t)h->max_updates);
    ALLOC(h->Tu, (size_t)h->max_updates);
    ALLOC(h->skipu, (size_t)h->max_updates);
    ALLOC(h->tauC, (size_t)kMaxT);
    ALLOC(h->tauD, (size_t)kMaxT);
    ALLOC(h->tau_old, (size_t)kMaxT);
    ALLOC(h->tauC_hist, t * h->max_updates);
    ALLOC(h->tauD_hist, t * h->max_updates);
    ALLOC(h->J, (size_t)kMaxT);
    ALLOC(h->J_hist, t * h->max_updates);
    ALLOC(h->G, t * t);
    ALLOC(h->gpart, (size_t)h->gslabs * h->gld * h->gld);
    if (h->gram_merge) ALLOC(h->grun, (size_t)1);
    ALLOC(h->QR, ell * t * cg);
    ALLOC(h->qr_tau, (size_t)kMaxT * cg);
    ALLOC(h->P, t * h->n_max);
    if (cg > 1 && h->t > kAlg4Gemm) ALLOC(h->Pz, t * h->n_max * cg);
    ALLOC(h->SSTk, ell * ell * h->nzmax);
    ALLOC(h->Qm, ell * t * cg);
    ALLOC(h->Mm, t * ell * cg);
    ALLOC(h->Y, ell * t * cg);
    ALLOC(h->PPt, t * t * cg);
    ALLOC(h->hw, hutch_work_doubles(h->ell, h->t) * cg);
    ALLOC(h->colptr_dev, (size_t)h->n_max);
    ALLOC(h->slot_ptr, (size_t)t);
    ALLOC(h->normpart, (size_t)h->n_slabs * h->b_max);
    ALLOC(h->sc, (size_t)1);
    ALLOC(h->sc_hist, (size_t)h->max_updates);
    ALLOC(h->Ghist, t * t * h->max_updates);
    if (h->best4) {
      ALLOC(h->b4_Pc, 4 * t * h->n_max);
      ALLOC(h->b4_Pprev, t * h->n_max);
      ALLOC(h->b4_M5, t * ell);
      ALLOC(h->b4_L, t * t);
      ALLOC(h->b4_T, t * t);
      ALLOC(h->b4_rA, ell * h->n_max);
      ALLOC(h->b4_D6, t * h->n_max);
      ALLOC(h->b4_QR6, ell * t);
      ALLOC(h->b4_tau6, (size_t)kMaxT);
      ALLOC(h->b4_Qm6, ell * t);
      ALLOC(h->b4_Mm6, t * ell);
      ALLOC(h->b4_Xc, t * t * h->nzmax);
      ALLOC(h->b4_sc6, (size_t)1);
      ALLOC(h->b4_rec, (size_t)1);
      ALLOC(h->b4_recq, 4 * (size_t)h->max_updates);
      ALLOC(h->b4_qstar, (size_t)h->max_updates);
    }
    ALLOC(h->recs, (size_t)h->max_updates);
    if ((st = dalloc(h, &h->part, (size_t)h->n_slabs * h->b_max * h->ell_pad * psize)) != RID_OK)
      goto fail_alloc;
    if ((st = dalloc(h, &h->cpool, (size_t)h->ldc * t * h->esize)) != RID_OK) goto fail_alloc;
  }
#undef ALLOC
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->side_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->coeff_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->colptr_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    st = fail(nullptr, RID_EDEVICE, "side stream creation failed");
    goto fail_alloc;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&h->colptr_host), sizeof(uint64_t) * h->n_max,
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    st = fail(nullptr, RID_ENOMEM, "pinned host allocation failed");
    goto fail_alloc;
  }
  if (h->cgroup > 1 && !member) {
    // at most 16 launches per coefficient phase, each with a table of cgroup
    // argument blocks and grid sizes
    h->ctab_cap = 16 * ((size_t)h->cgroup * (sizeof(UpdArgs) + sizeof(int4)) + 512);
    if ((st = dalloc(h, reinterpret_cast<void**>(&h->ctab_dev), h->ctab_cap)) != RID_OK) goto fail_alloc;
    for (int i = 0; i < rid_stream::kTabSlots; ++i)
      if (hipHostMalloc(reinterpret_cast<void**>(&h->ctab_host[i]), h->ctab_cap, hipHostMallocDefault) != hipSuccess ||
          hipEventCreateWithFlags(&h->ctab_ev[i], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(nullptr, RID_ENOMEM, "pinned host allocation failed");
        goto fail_alloc;
      }
  }
  if (hipMemsetAsync(h->cpool, 0, (size_t)h->ldc * t * h->esize, h->s) != hipSuccess ||
      hipMemsetAsync(h->SST[0], 0, ell * ell * 8, h->s) != hipSuccess ||
      hipMemsetAsync(h->G, 0, t * t * 8, h->s) != hipSuccess ||
      hipMemsetAsync(h->recs, 0, sizeof(rid_update) * h->max_updates, h->s) != hipSuccess) {
    st = fail(nullptr, RID_EDEVICE, "hipMemsetAsync failed");
    goto fail_alloc;
  }
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(kMaxT), 0, h->s, h->J, h->tau_old, h->t, h->sc,
                     h->slot_ptr, static_cast<const char*>(h->cpool), (int64_t)h->ldc * h->esize);
  if (hipGetLastError() != hipSuccess) {
    st = fail(nullptr, RID_EDEVICE, "init kernel launch failed");
    goto fail_alloc;
  }
  *out = h;
  return RID_OK;
fail_alloc:
  g_last_err = h->last_err.empty() ? g_last_err : h->last_err;
  free_all(h);
  delete h;
  return st;
}

// ---------------------------------------------------------------------------
// internal stream operations
// ---------------------------------------------------------------------------
static hipEvent_t take_event(rid_stream* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Starts a timed interval on the handle's stream (no-op unless profiling).
static int mark_begin(rid_stream* h, int kind, double bytes, hipStream_t on = nullptr, int64_t aux = -1) {
  if (!h->profiling) return -1;
  rid_stream::Mark mk{take_event(h), take_event(h), kind, bytes, on ? on : h->s, aux};
  if (!mk.a || !mk.b || hipEventRecord(mk.a, mk.on) != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  h->marks.push_back(mk);
  return (int)h->marks.size() - 1;
}

static void mark_end(rid_stream* h, int idx) {
  if (idx < 0) return;
  if (hipEventRecord(h->marks[idx].b, h->marks[idx].on) != hipSuccess) (void)hipGetLastError();
}

// Work enqueued on the handle's stream after this call also waits for the
// side stream's work so far.
static rid_status join_side(rid_stream* h) {
  if (!h->side_used) return RID_OK;
  RID_HIP(h, hipEventRecord(h->side_ev, h->side));
  RID_HIP(h, hipStreamWaitEvent(h->s, h->side_ev, 0));
  h->side_used = false;
  return RID_OK;
}
static rid_status upload_colptrs(rid_stream* h) {
  if (h->n_uploaded < h->n_pushed) {
    const int64_t n = h->n_pushed - h->n_uploaded;
    RID_HIP(h, hipMemcpyAsync(h->colptr_dev + h->n_uploaded, h->colptr_host + h->n_uploaded,
                              n * sizeof(uint64_t), hipMemcpyHostToDevice, h->s));
    RID_HIP(h, hipEventRecord(h->colptr_ev, h->s));
    h->colptr_pending = true;
    h->n_uploaded = h->n_pushed;
  }
  return RID_OK;
}

static SketchArgs sketch_args(rid_stream* h, int64_t c0, int b) {
  SketchArgs a;
  a.colptr = h->colptr_dev;
  a.c0 = c0;
  a.b = b;
  a.b_max = h->b_max;
  a.m = h->m;
  a.slab_rows = h->slab_rows;
  a.n_slabs = h->n_slabs;
  a.n_mt = h->n_mt;
  a.n_nt = (b + h->cols_per_wg - 1) / h->cols_per_wg;
  a.ell_pad = h->ell_pad;
  a.ell = h->ell;
  a.rbw = h->rbw;
  a.wide = h->wide;
  a.seed = h->cfg.omega_seed;
  a.part = h->part;
  a.normpart = h->normpart;
  a.S = h->S;
  a.colsq = h->colsq;
  a.nonfinite = &h->sc->nonfinite;
  return a;
}

static rid_status sketch_range(rid_stream* h, int64_t c0, int b) {
  const SketchArgs a = sketch_args(h, c0, b);
  int mk = mark_begin(h, 0, (double)b * (double)h->m * h->esize);
  RID_HIP(h, launch_sketch(h->prec, a, h->s));
  mark_end(h, mk);
  if (h->reduce_wait) {
    RID_HIP(h, hipStreamWaitEvent(h->s, h->coeff_ev, 0));
    h->reduce_wait = false;
  }
  mk = mark_begin(h, 1, 0.0);
  RID_HIP(h, launch_sketch_reduce(h->prec, a, h->s));
  mark_end(h, mk);
  return RID_OK;
}

// Enqueues updates n_updates .. n_updates + nz - 1: n_full of t columns and,
// when last > 0, one more of `last` columns.
static BatchArgs batch_args(rid_stream* h, int n_full, int last) {
  const int nz = n_full + (last > 0 ? 1 : 0);
  BatchArgs b;
  b.ell = h->ell;
  b.k = h->k;
  b.t = h->t;
  b.nz = nz;
  b.u0 = h->n_updates;
  b.c0 = h->n_updates * h->t;
  b.total = (int64_t)n_full * h->t + last;
  b.ridge_floor = h->cfg.ridge_floor;
  b.S = h->S;
  b.colsq = h->colsq;
  b.sst_in = h->SST[h->sst_cur];
  b.sst_out = h->SST[h->sst_cur ^ 1];
  b.sst_keep = h->SSTk;
  b.W = h->W;
  b.hv = h->hv;
  b.Fu = h->Fu;
  b.tru = h->Tu;
  b.skipu = h->skipu;
  b.recs = h->recs;
  return b;
}

// 32 x 32 tiles of the split Gram of a list of nj columns whose first nq are
// new (the new-against-new tiles below the diagonal are not formed).
static int gram_tiles(int nq, int nj) {
  const int TQ = (nq + 31) / 32, TJ = (nj + 31) / 32;
  int n = 0;
  for (int r = 0; r < TQ; ++r) n += TJ - std::min(r, nq / 32);
  return n;
}

// Arguments of update n_updates + z of a batch of n_full full updates.
static UpdArgs upd_args(rid_stream* h, int z, int n_full, int last) {
  UpdArgs a;
  {
    a.ell = h->ell;
    a.k = h->k;
    a.t = h->t;
    a.n1 = h->n1;
    a.n2 = h->n2;
    a.u = h->n_updates + z;
    a.c0 = a.u * h->t;
    a.cnt = (z < n_full) ? h->t : last;
    a.n_obs = a.c0 + a.cnt;
    a.fill_mult = h->fill_mult;
    a.ridge_floor = h->cfg.ridge_floor;
    a.select_seed = h->cfg.select_seed;
    a.m = h->m;
    a.ldc = h->ldc;
    a.data_f64 = h->data_f64;
    a.gram_split = h->gram_split ? 1 : 0;
    a.S = h->S;
    a.SSTu = h->SSTk + (size_t)z * h->ell * h->ell;
    a.colsq = h->colsq;
    a.W = h->W + (size_t)z * h->ell * h->ell;
    a.hv = h->hv + (size_t)z * 6 * h->ell;
    a.Qs = h->Qs + (size_t)z * h->ell * h->ell;
    a.Ys = h->Ys + (size_t)z * h->ell * 2 * h->t;
    a.Fu = h->Fu;
    a.skipu = h->skipu;
    a.J = h->J;
    a.tau_old = h->tau_old;
    a.tauC = h->tauC;
    a.tauD = h->tauD;
    a.J_hist = h->J_hist;
    a.tauC_hist = h->tauC_hist;
    a.tauD_hist = h->tauD_hist;
    a.colptr = h->colptr_dev;
    a.cpool = h->cpool;
    a.slot_ptr = h->slot_ptr;
    a.flush_last = 0;
    a.G = h->G;
    a.gpart = h->gpart;
    a.gld = h->gld;
    a.grun = nullptr;
    a.grun_u = 0;
    a.gslabs = h->gslabs;
    a.gslab_rows = h->gslab_rows;
    a.QR = h->QR;
    a.qr_tau = h->qr_tau;
    a.P = h->P;
    a.Qm = h->Qm;
    a.Mm = h->Mm;
    a.Y = h->Y;
    a.PPt = h->PPt;
    a.hw = h->hw;
    a.sc = h->sc;
    a.recs = h->recs;
  }
  return a;
}

// Buffers of the coefficient phase of update z of a flush of nz updates: slice
// z % cgroup of the per-update scratch.  P in place for the last update (the
// one rid_coefficients reads); the others form P only above kAlg4Gemm, in a
// slice of Pz.
static void coeff_slice(rid_stream* h, UpdArgs& a, int z, int nz) {
  const size_t zz = (size_t)(z % h->cgroup), ell = h->ell, t = h->t;
  a.QR = h->QR + zz * ell * t;
  a.qr_tau = h->qr_tau + zz * kMaxT;
  a.Qm = h->Qm + zz * ell * t;
  a.Mm = h->Mm + zz * t * ell;
  a.Y = h->Y + zz * ell * t;
  a.PPt = h->PPt + zz * t * t;
  a.hw = h->hw + zz * hutch_work_doubles(h->ell, h->t);
  a.P = (z == nz - 1 || !h->Pz) ? h->P : h->Pz + zz * t * (size_t)h->n_max;
}

// The next pinned host slot for argument tables (its previous copy done).
static rid_status take_table(rid_stream* h, Stage& stg) {
  h->ctab_slot = (h->ctab_slot + 1) % rid_stream::kTabSlots;
  if (h->ctab_used[h->ctab_slot]) RID_HIP(h, hipEventSynchronize(h->ctab_ev[h->ctab_slot]));
  stg.host = h->ctab_host[h->ctab_slot];
  stg.dev = h->ctab_dev;
  stg.cap = h->ctab_cap;
  stg.used = 0;
  stg.overflow = false;
  return RID_OK;
}

// Algs. 5-7 buffers of update u (slot z of the flush).
static B4Args b4_args(rid_stream* h, int64_t u, int z) {
  const size_t t = h->t;
  B4Args b;
  b.n_prev = u * h->t;   // every update before the last of a stream is full
  b.J_prev = u > 0 ? h->J_hist + (u - 1) * t : nullptr;
  b.G_prev = u > 0 ? h->Ghist + (u - 1) * t * t : nullptr;
  b.Xc = h->b4_Xc + (size_t)z * t * t;
  b.Pc = h->b4_Pc;
  b.Pprev = h->b4_Pprev;
  b.Pout = h->P;
  b.M5 = h->b4_M5;
  b.L = h->b4_L;
  b.T = h->b4_T;
  b.rA = h->b4_rA;
  b.D6 = h->b4_D6;
  b.QR6 = h->b4_QR6;
  b.tau6 = h->b4_tau6;
  b.Qm6 = h->b4_Qm6;
  b.Mm6 = h->b4_Mm6;
  b.sc6 = h->b4_sc6;
  b.scratch_rec = h->b4_rec;
  b.recq = h->b4_recq + 4 * u;
  b.qstar = h->b4_qstar + u;
  b.n_max = h->n_max;
  return b;
}

static rid_status run_updates(rid_stream* h, int n_full, int last) {
  const int nz = n_full + (last > 0 ? 1 : 0);
  if (nz == 0) return RID_OK;
  if (nz > h->nzmax) return fail(h, RID_EDEVICE, "internal: update batch larger than its slots");
  std::vector<UpdArgs> co(nz);
  const BatchArgs b = batch_args(h, n_full, last);
  if (h->coeff_pending) RID_HIP(h, hipStreamWaitEvent(h->s, h->coeff_ev, 0));
  int mk = mark_begin(h, 2, 0.0);
  RID_HIP(h, launch_update_batch(b, h->s));
  // Q of each update depends on its tridiagonalisation only
  RID_HIP(h, launch_update_q_all(upd_args(h, 0, n_full, last), nz, h->s));
  mark_end(h, mk);
  h->sst_cur ^= 1;
  const int64_t flush_c0 = upd_args(h, 0, n_full, last).c0;  // first column the flush scans
  // Alg. 4 and Alg. 8 of each update read snapshots of the selection state
  // (the next update's selection rewrites J, G and the slot lists)
  auto hist = [&](const UpdArgs& x, int zz) {
    UpdArgs ac = x;
    ac.sc = h->sc_hist + x.u;
    ac.G = h->Ghist + (size_t)x.u * h->t * h->t;
    ac.J = h->J_hist + (size_t)x.u * h->t;
    coeff_slice(h, ac, zz, nz);
    if (h->best4) ac.P = h->b4_Pc;   // Alg. 4's candidate
    return ac;
  };
  int z = 0;
  if (h->gram_merge && nz > 1) {
    // Every selection of the flush first (none reads a Gram entry), each
    // state kept; then the split Grams of runs of consecutive updates (the
    // last excepted: its Gram copies the basis into the pool), a run growing
    // while its list [new at each update, the others occupied at its first]
    // fits one workgroup's tiles, so that the run reads each column once.
    std::vector<UpdArgs> A(nz);
    for (int zz = 0; zz < nz; ++zz) {
      A[zz] = upd_args(h, zz, n_full, last);
      A[zz].flush_last = zz == nz - 1;
      mk = mark_begin(h, 2, (double)A[zz].u);
      RID_HIP(h, launch_update_select(A[zz], h->s, false));
      mark_end(h, mk);
      if (zz < nz - 1) {
        const UpdArgs ac = hist(A[zz], zz);
        RID_HIP(h, launch_update_snapshot(A[zz], ac.sc, ac.G, h->s));  // its state; G follows its Gram
      }
    }
    std::vector<rid_update> R(nz);
    RID_HIP(h, hipMemcpyAsync(R.data(), h->recs + A[0].u, sizeof(rid_update) * nz, hipMemcpyDeviceToHost, h->s));
    RID_HIP(h, hipStreamSynchronize(h->s));
    while (z < nz - 1) {
      int zb = z, nq = R[z].n_filled, nj = R[z].n_occupied;
      while (zb + 1 < nz - 1 && zb + 2 - z <= kGramRunMax) {
        const int nq2 = nq + R[zb + 1].n_filled, nj2 = nj + R[zb + 1].n_filled;
        if (nj2 > kGramRunCols || gram_tiles(nq2, nj2) > kGramRunTiles) break;
        nq = nq2;
        nj = nj2;
        ++zb;
      }
      const int nu = zb - z + 1;
      mk = mark_begin(h, 3, nq > 0 ? (double)nj * (double)h->m * h->esize : 0.0, nullptr, -2);
      if (mk >= 0) h->marks[mk].nu = nu;
      RID_HIP(h, launch_update_gram_run(A[zb], nu, nq, nj, h->sc_hist, h->J_hist, h->grun, h->s));
      for (int w = 0; w < nu; ++w) {
        const UpdArgs ac = hist(A[z + w], z + w);
        UpdArgs aw = A[z + w];
        aw.sc = ac.sc;
        aw.J = ac.J;
        RID_HIP(h, launch_update_gram_run_entries(aw, w, h->grun, h->s));
        RID_HIP(h, launch_update_snapshot(aw, ac.sc, ac.G, h->s));
        co[z + w] = ac;
      }
      mark_end(h, mk);
      h->last_nobs = A[zb].n_obs;
      z = zb + 1;
    }
    // the last update: its Gram on the running state, as below
    UpdArgs a = A[z];
    mk = mark_begin(h, 3, (double)a.u, nullptr, flush_c0);
    RID_HIP(h, launch_update_gram(a, h->s));
    mark_end(h, mk);
    const UpdArgs ac = hist(a, z);
    co[z] = ac;
    RID_HIP(h, launch_update_snapshot(a, ac.sc, ac.G, h->s));
    h->last_nobs = a.n_obs;
    z = nz;
  }
  for (; z < nz;) {
    UpdArgs a = upd_args(h, z, n_full, last);
    a.flush_last = z == nz - 1;
    mk = mark_begin(h, 2, (double)a.u);
    RID_HIP(h, launch_update_select(a, h->s, false));
    mark_end(h, mk);
    mk = mark_begin(h, 3, (double)a.u, nullptr, a.flush_last ? flush_c0 : -1);
    // Alg. 7 needs the new columns' products with the pruned ones, which the
    // Gram's pool copy overwrites
    if (h->best4 && a.u > 0) RID_HIP(h, launch_best4_cross(a, b4_args(h, a.u, z), h->s));
    RID_HIP(h, launch_update_gram(a, h->s));
    mark_end(h, mk);
    const UpdArgs ac = hist(a, z);
    co[z] = ac;
    RID_HIP(h, launch_update_snapshot(a, ac.sc, ac.G, h->s));
    h->last_nobs = a.n_obs;
    ++z;
  }
  // The coefficient phases of the flush, on the side stream once the last
  // snapshot is taken: each is a chain of small latency-bound kernels (one
  // workgroup for either QR), so the updates of a group share every launch.
  RID_HIP(h, hipEventRecord(h->side_ev, h->s));
  RID_HIP(h, hipStreamWaitEvent(h->side, h->side_ev, 0));
  mk = mark_begin(h, 4, (double)h->n_updates, h->side);
  for (int z0 = 0; z0 < nz; z0 += h->cgroup) {
    const int g = std::min(h->cgroup, nz - z0);
    if (g == 1) {
      RID_HIP(h, launch_update_coeff(co[z0], h->side, h->best4 || z0 == nz - 1));
      if (h->best4) RID_HIP(h, launch_best4(co[z0], b4_args(h, co[z0].u, z0), h->side));
      continue;
    }
    Stage stg;
    rid_status sts = take_table(h, stg);
    if (sts != RID_OK) return sts;
    std::vector<BLaunch> L;
    std::unique_ptr<bool[]> want_p(new bool[g]);
    for (int q = 0; q < g; ++q) want_p[q] = (z0 + q == nz - 1);
    plan_update_coeff_b(co.data() + z0, g, stg, L, want_p.get());
    if (stg.overflow) return fail(h, RID_EDEVICE, "internal: coefficient tables exceed their staging buffer");
    RID_HIP(h, hipMemcpyAsync(h->ctab_dev, stg.host, stg.used, hipMemcpyHostToDevice, h->side));
    RID_HIP(h, hipEventRecord(h->ctab_ev[h->ctab_slot], h->side));
    h->ctab_used[h->ctab_slot] = true;
    RID_HIP(h, run_launches(L, h->side));
  }
  RID_HIP(h, hipEventRecord(h->coeff_ev, h->side));
  h->coeff_pending = true;
  mark_end(h, mk);
  h->side_used = true;
  h->n_updates += nz;
  return RID_OK;
}

// Sketch every pushed column (in batches of at most b_max) and enqueue every
// update whose t columns are sketched.
static rid_status flush_all(rid_stream* h) {
  rid_status st = upload_colptrs(h);
  if (st != RID_OK) return st;
  while (h->n_sketched < h->n_pushed) {
    const int b = (int)std::min<int64_t>(h->b_max, h->n_pushed - h->n_sketched);
    if ((st = sketch_range(h, h->n_sketched, b)) != RID_OK) return st;
    h->n_sketched += b;
    const int full = (int)(h->n_sketched / h->t - h->n_updates);
    if ((st = run_updates(h, full, 0)) != RID_OK) return st;
  }
  return RID_OK;
}

// Sketch full batches of the lookahead once more than a batch is pending
// (used after pushes).  A batch that is exactly full waits for the next push
// or for finalize, so that a final partial update can share its eigen-solve
// launch with the full updates of that batch.
static rid_status flush_full(rid_stream* h) {
  rid_status st = RID_OK;
  if (h->n_pushed - h->n_sketched <= h->b_max) return RID_OK;
  if ((st = upload_colptrs(h)) != RID_OK) return st;
  while (h->n_pushed - h->n_sketched > h->b_max) {
    if ((st = sketch_range(h, h->n_sketched, h->b_max)) != RID_OK) return st;
    h->n_sketched += h->b_max;
    const int full = (int)(h->n_sketched / h->t - h->n_updates);
    if ((st = run_updates(h, full, 0)) != RID_OK) return st;
  }
  return RID_OK;
}

static rid_status sync_check(rid_stream* h) {
  rid_status st = join_side(h);
  if (st != RID_OK) return st;
  RID_HIP(h, hipStreamSynchronize(h->s));
  int32_t nf = 0;
  RID_HIP(h, hipMemcpy(&nf, &h->sc->nonfinite, sizeof(nf), hipMemcpyDeviceToHost));
  if (nf) return fail(h, RID_ENUMERIC, "non-finite snapshot value");
  return RID_OK;
}

extern "C" {

static rid_status push_columns(rid_stream* h, const void* d_cols, int64_t ld, int32_t b, uint32_t flags,
                               bool flush);

rid_status rid_push_snapshots(rid_stream* h, const void* d_cols, int64_t ld, int32_t b, uint32_t flags) {
  if (!h) return fail(nullptr, RID_EINVAL, "null handle");
  if (h->owner) return fail(h, RID_ESTATE, "the stream belongs to a batch: push through rid_push_batch");
  return push_columns(h, d_cols, ld, b, flags, true);
}

}  // extern "C"

// Appends b columns to the stream's column table (BORROW) or ring (COPY).
// With `flush`, full lookahead batches are sketched and their updates
// enqueued as they complete; a batch member leaves that to the batch.
static rid_status batch_make_room(rid_batch* bt);

static rid_status push_columns(rid_stream* h, const void* d_cols, int64_t ld, int32_t b, uint32_t flags,
                               bool flush) {
  if (h->failed || h->finalized) return fail(h, RID_ESTATE, "stream finalized or failed");
  if (b < 0 || ld < h->m || (b > 0 && !d_cols) || (flags != RID_COPY && flags != RID_BORROW))
    return fail(h, RID_EINVAL, "bad push arguments");
  if (b == 0) return RID_OK;
  if (h->n_pushed + b > h->n_max) return fail(h, RID_ECAPACITY, "push exceeds n_max");
  const uintptr_t base = reinterpret_cast<uintptr_t>(d_cols);
  const int64_t es = h->esize;
  rid_status st;
  if (flags == RID_BORROW) {
    if (base % 16 != 0 || (ld * es) % 16 != 0)
      return fail(h, RID_EINVAL, "BORROW needs 16-byte aligned columns (pointer and ld * size)");
    for (int j = 0; j < b; ++j) h->colptr_host[h->n_pushed + j] = base + (uint64_t)j * ld * es;
    h->n_pushed += b;
    return flush ? flush_full(h) : RID_OK;
  }
  // COPY: stage the columns in the ring, never overwriting a column that an
  // enqueued update has not consumed yet.
  if (!h->ring) {
    h->ring_cap = std::max<int64_t>(h->b_max, 2 * (int64_t)h->t);
    h->ring_cap = (h->ring_cap + h->t - 1) / h->t * h->t;
    h->ring_ld = h->ldc;
    if ((st = dalloc(h, &h->ring, (size_t)h->ring_cap * h->ring_ld * es)) != RID_OK) return st;
  }
  int done = 0;
  while (done < b) {
    const int64_t consumed = h->n_updates * h->t;
    int64_t space = h->ring_cap - (h->n_pushed - consumed);
    if (space <= 0) {
      if ((st = (h->owner ? batch_make_room(h->owner) : flush_all(h))) != RID_OK) return st;
      if (h->failed) return fail(h, RID_ESTATE, "stream failed");
      continue;
    }
    const int64_t slot = h->n_pushed % h->ring_cap;
    int64_t chunk = std::min<int64_t>({(int64_t)(b - done), space, h->ring_cap - slot});
    char* dst = reinterpret_cast<char*>(h->ring) + slot * h->ring_ld * es;
    const char* src = reinterpret_cast<const char*>(d_cols) + (int64_t)done * ld * es;
    RID_HIP(h, hipMemcpy2DAsync(dst, h->ring_ld * es, src, ld * es, h->m * es, chunk,
                                hipMemcpyDeviceToDevice, h->s));
    for (int64_t j = 0; j < chunk; ++j)
      h->colptr_host[h->n_pushed + j] = reinterpret_cast<uint64_t>(dst) + (uint64_t)j * h->ring_ld * es;
    h->n_pushed += chunk;
    done += (int)chunk;
    if (flush && (h->n_pushed - h->n_sketched >= h->b_max || h->n_pushed - consumed >= h->ring_cap))
      if ((st = flush_all(h)) != RID_OK) return st;
  }
  return RID_OK;
}

extern "C" {

rid_status rid_flush(rid_stream* h) {
  if (!h) return fail(nullptr, RID_EINVAL, "null handle");
  if (h->failed) return fail(h, RID_ESTATE, "stream failed");
  return flush_all(h);
}

rid_status rid_finalize(rid_stream* h) {
  if (!h) return fail(nullptr, RID_EINVAL, "null handle");
  if (h->owner) return fail(h, RID_ESTATE, "the stream belongs to a batch: use rid_finalize_batch");
  if (h->failed || h->finalized) return fail(h, RID_ESTATE, "stream finalized or failed");
  // Sketch what is left; the full updates completed by the last sketch launch
  // share one batch (one eigen-solve launch) with the final partial update.
  rid_status st = upload_colptrs(h);
  if (st != RID_OK) return st;
  while (h->n_sketched < h->n_pushed) {
    const int b = (int)std::min<int64_t>(h->b_max, h->n_pushed - h->n_sketched);
    if ((st = sketch_range(h, h->n_sketched, b)) != RID_OK) return st;
    h->n_sketched += b;
    if (h->n_sketched < h->n_pushed) {
      const int full = (int)(h->n_sketched / h->t - h->n_updates);
      if ((st = run_updates(h, full, 0)) != RID_OK) return st;
    }
  }
  const int full = (int)(h->n_pushed / h->t - h->n_updates);
  const int64_t rem = h->n_pushed - (h->n_updates + full) * h->t;
  if ((full > 0 || rem > 0) && (st = run_updates(h, full, (int)rem)) != RID_OK) return st;
  h->finalized = true;
  return RID_OK;
}

static rid_status reset_stream(rid_stream* h);

rid_status rid_reset(rid_stream* h) {
  if (!h) return fail(nullptr, RID_EINVAL, "null handle");
  if (h->owner) return fail(h, RID_ESTATE, "the stream belongs to a batch");
  return reset_stream(h);
}

}  // extern "C"

// Without a host wait for the device: the state is cleared in stream order
// behind the previous pass, so the host can enqueue the next pass meanwhile;
// it only waits until the last upload of the pinned column-pointer table has
// been copied, since the next pushes rewrite that table from the start.  The
// previous pass's coefficient phases may still run on the second stream: they
// read snapshots, kept copies of SS^T and S, and write the records, P and
// their own buffers.  The records are cleared behind them on that stream; the
// next sketch reduction (S) and the next update (snapshots, SS^T, records)
// wait for them, so the next pass's sketch overlaps them.
static rid_status reset_stream(rid_stream* h) {
  if (h->failed) return fail(h, RID_ESTATE, "stream failed");
  const size_t ell = h->ell, t = h->t;
  if (h->side_used && !h->owner) {
    RID_HIP(h, hipMemsetAsync(h->recs, 0, sizeof(rid_update) * h->max_updates, h->side));
    RID_HIP(h, hipEventRecord(h->coeff_ev, h->side));
    h->coeff_pending = true;
    h->reduce_wait = true;
  } else {
    rid_status st = join_side(h);
    if (st != RID_OK) return st;
    RID_HIP(h, hipMemsetAsync(h->recs, 0, sizeof(rid_update) * h->max_updates, h->s));
  }
  if (h->colptr_pending) RID_HIP(h, hipEventSynchronize(h->colptr_ev));
  h->colptr_pending = false;
  h->sst_cur = 0;
  RID_HIP(h, hipMemsetAsync(h->SST[0], 0, ell * ell * 8, h->s));
  RID_HIP(h, hipMemsetAsync(h->G, 0, t * t * 8, h->s));
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(kMaxT), 0, h->s, h->J, h->tau_old, h->t, h->sc,
                     h->slot_ptr, static_cast<const char*>(h->cpool), (int64_t)h->ldc * h->esize);
  RID_HIP(h, hipGetLastError());
  h->n_pushed = h->n_sketched = h->n_uploaded = h->n_updates = h->last_nobs = 0;
  h->finalized = false;
  return RID_OK;
}

extern "C" {

static rid_status getter_prologue(rid_stream* h) {
  if (h->failed) return fail(h, RID_ESTATE, "stream failed");
  rid_status st = flush_all(h);
  if (st != RID_OK) return st;
  return sync_check(h);
}

rid_status rid_select(rid_stream* h, int64_t* J, int32_t cap, int32_t* t_out) {
  if (!h || !J || !t_out) return fail(h, RID_EINVAL, "null argument");
  if (cap < h->t) return fail(h, RID_EINVAL, "cap < t");
  rid_status st = getter_prologue(h);
  if (st != RID_OK) return st;
  if (h->n_updates == 0) return fail(h, RID_ESTATE, "no update has run yet");
  RID_HIP(h, hipMemcpy(J, h->J, sizeof(int64_t) * h->t, hipMemcpyDeviceToHost));
  *t_out = h->t;
  return RID_OK;
}

rid_status rid_coefficients(rid_stream* h, double* P, int64_t ldp, int64_t cap_cols, int64_t* n_cols,
                            uint32_t where) {
  if (!h || !P || !n_cols) return fail(h, RID_EINVAL, "null argument");
  if (ldp < h->t || (where != RID_HOST && where != RID_DEVICE)) return fail(h, RID_EINVAL, "bad ldp or where");
  rid_status st = getter_prologue(h);
  if (st != RID_OK) return st;
  if (h->n_updates == 0) return fail(h, RID_ESTATE, "no update has run yet");
  if (cap_cols < h->last_nobs) return fail(h, RID_EINVAL, "cap_cols smaller than the covered columns");
  *n_cols = h->last_nobs;
  RID_HIP(h, hipMemcpy2D(P, ldp * 8, h->P, (size_t)h->t * 8, (size_t)h->t * 8, h->last_nobs,
                         where == RID_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice));
  return RID_OK;
}

rid_status rid_error_estimate(rid_stream* h, rid_error* e) {
  if (!h || !e) return fail(h, RID_EINVAL, "null argument");
  rid_status st = getter_prologue(h);
  if (st != RID_OK) return st;
  if (h->n_updates == 0) return fail(h, RID_ESTATE, "no update has run yet");
  rid_update r;
  RID_HIP(h, hipMemcpy(&r, h->recs + (h->n_updates - 1), sizeof(r), hipMemcpyDeviceToHost));
  e->E2 = r.E2;
  e->E_abs = sqrt(r.E2 > 0.0 ? r.E2 : 0.0);
  e->rel = r.F > 0.0 ? e->E_abs / sqrt(r.F) : 0.0;
  e->F = r.F;
  e->n_obs = r.n_obs;
  e->update = r.update;
  return RID_OK;
}

rid_status rid_reconstruct(rid_stream* h, int64_t j0, int32_t c, void* d_out, int64_t ld) {
  if (!h || (!d_out && c > 0)) return fail(h, RID_EINVAL, "null argument");
  if (h->failed) return fail(h, RID_ESTATE, "stream failed");
  if (h->n_updates == 0) return fail(h, RID_ESTATE, "no update has run yet");
  if (j0 < 0 || c < 0 || j0 + c > h->last_nobs || ld < h->m)
    return fail(h, RID_EINVAL, "columns outside the covered range or ld < m");
  if (c == 0) return RID_OK;
  rid_status jst = join_side(h);  // P of the last update comes from the side stream
  if (jst != RID_OK) return jst;
  dim3 grid((unsigned)((h->m + 255) / 256), (unsigned)((c + 15) / 16));
  if (h->data_f64)
    hipLaunchKernelGGL(reconstruct_kernel<double>, grid, dim3(256), 0, h->s,
                       reinterpret_cast<const double*>(h->cpool), h->ldc, h->P, h->t, h->J, h->m, j0, c,
                       reinterpret_cast<double*>(d_out), ld);
  else
    hipLaunchKernelGGL(reconstruct_kernel<float>, grid, dim3(256), 0, h->s,
                       reinterpret_cast<const float*>(h->cpool), h->ldc, h->P, h->t, h->J, h->m, j0, c,
                       reinterpret_cast<float*>(d_out), ld);
  RID_HIP(h, hipGetLastError());
  if (h->owner) {  // a batch member: the caller's stream (possibly the null stream) waits for the result
    RID_HIP(h, hipEventRecord(h->join_ev, h->s));
    RID_HIP(h, hipStreamWaitEvent(h->join, h->join_ev, 0));
  }
  return RID_OK;
}

rid_status rid_get_coeff_choice(rid_stream* h, int64_t u, double* e2, int32_t* q_star) {
  if (!h || !e2 || !q_star) return fail(h, RID_EINVAL, "null argument");
  if (!h->best4) return fail(h, RID_ESTATE, "the stream does not run RID_COEFF_BEST4");
  rid_status st = getter_prologue(h);
  if (st != RID_OK) return st;
  if (u < 0 || u >= h->n_updates) return fail(h, RID_EINVAL, "update index out of range");
  rid_update rq[4];
  RID_HIP(h, hipMemcpy(rq, h->b4_recq + 4 * u, sizeof(rq), hipMemcpyDeviceToHost));
  RID_HIP(h, hipMemcpy(q_star, h->b4_qstar + u, sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int q = 0; q < 4; ++q) e2[q] = rq[q].E2;
  return RID_OK;
}

rid_status rid_get_info(rid_stream* h, rid_info* info) {
  if (!h || !info) return fail(h, RID_EINVAL, "null argument");
  if (!h->failed) {
    hipError_t e = hipStreamSynchronize(h->side);
    if (e == hipSuccess) e = hipStreamSynchronize(h->s);
    if (e != hipSuccess) fail(h, RID_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  }
  info->n_pushed = h->n_pushed;
  info->n_sketched = h->n_sketched;
  info->n_updates = h->n_updates;
  info->release_watermark = h->failed ? 0 : std::min(h->n_updates * h->t, h->n_sketched);
  if (h->finalized && !h->failed) info->release_watermark = h->n_pushed;
  info->failed = h->failed ? 1 : 0;
  info->finalized = h->finalized ? 1 : 0;
  info->last_status = h->last_status;
  info->reserved0 = 0;
  info->device_bytes = (int64_t)h->dev_bytes;
  return RID_OK;
}

rid_status rid_get_update(rid_stream* h, int64_t u, rid_update* rec, int64_t* J_out, double* tau_C,
                          double* tau_D) {
  if (!h || !rec) return fail(h, RID_EINVAL, "null argument");
  rid_status st = getter_prologue(h);
  if (st != RID_OK) return st;
  if (u < 0 || u >= h->n_updates) return fail(h, RID_EINVAL, "update index out of range");
  RID_HIP(h, hipMemcpy(rec, h->recs + u, sizeof(*rec), hipMemcpyDeviceToHost));
  if (J_out) RID_HIP(h, hipMemcpy(J_out, h->J_hist + u * h->t, sizeof(int64_t) * h->t, hipMemcpyDeviceToHost));
  if (tau_C) RID_HIP(h, hipMemcpy(tau_C, h->tauC_hist + u * h->t, sizeof(double) * h->t, hipMemcpyDeviceToHost));
  if (tau_D) RID_HIP(h, hipMemcpy(tau_D, h->tauD_hist + u * h->t, sizeof(double) * rec->count, hipMemcpyDeviceToHost));
  return RID_OK;
}

rid_status rid_debug_state(rid_stream* h, double* S, int64_t lds, int64_t cap_cols, int64_t* n_cols,
                           double* colsq, double* G) {
  if (!h || !n_cols) return fail(h, RID_EINVAL, "null argument");
  rid_status st = getter_prologue(h);
  if (st != RID_OK) return st;
  *n_cols = h->n_sketched;
  if (S) {
    if (lds < h->ell || cap_cols < h->n_sketched) return fail(h, RID_EINVAL, "S too small");
    if (h->n_sketched > 0)
      RID_HIP(h, hipMemcpy2D(S, lds * 8, h->S, (size_t)h->ell * 8, (size_t)h->ell * 8, h->n_sketched,
                             hipMemcpyDeviceToHost));
  }
  if (colsq && h->n_sketched > 0)
    RID_HIP(h, hipMemcpy(colsq, h->colsq, sizeof(double) * h->n_sketched, hipMemcpyDeviceToHost));
  if (G) RID_HIP(h, hipMemcpy(G, h->G, sizeof(double) * h->t * h->t, hipMemcpyDeviceToHost));
  return RID_OK;
}

rid_status rid_profile_enable(rid_stream* h, int32_t on) {
  if (!h) return fail(nullptr, RID_EINVAL, "null handle");
  RID_HIP(h, hipStreamSynchronize(h->side));
  RID_HIP(h, hipStreamSynchronize(h->s));
  for (auto& mk : h->marks) {
    h->event_pool.push_back(mk.a);
    h->event_pool.push_back(mk.b);
  }
  h->marks.clear();
  h->profiling = on != 0;
  return RID_OK;
}

rid_status rid_profile_read(rid_stream* h, rid_profile* p) {
  if (!h || !p) return fail(h, RID_EINVAL, "null argument");
  RID_HIP(h, hipStreamSynchronize(h->side));
  RID_HIP(h, hipStreamSynchronize(h->s));
  memset(p, 0, sizeof(*p));
  for (auto& mk : h->marks) {
    float ms = 0.0f;
    RID_HIP(h, hipEventElapsedTime(&ms, mk.a, mk.b));
    switch (mk.kind) {
      case 0: p->sketch_ms += ms; p->sketch_launches += 1; p->sketch_bytes += mk.bytes; break;
      case 1: p->reduce_ms += ms; break;
      case 2: p->update_ms += ms; break;
      case 4: p->coeff_ms += ms; break;
      default: {
        // an update that brings new columns reads every occupied basis column
        // once (the new ones from the snapshots, the others from the pool)
        // and writes the new ones into the pool
        if (mk.aux == -2) {
          // a run of updates' Grams in one pass: its list's columns, read once
          p->update_ms += ms;
          p->updates += mk.nu;
          p->gram_ms += ms;
          if (mk.bytes > 0) {
            p->gram_bytes += mk.bytes;
            p->gram_launches += 1;
          }
          break;
        }
        rid_update r;
        RID_HIP(h, hipMemcpy(&r, h->recs + (int64_t)mk.bytes, sizeof(r), hipMemcpyDeviceToHost));
        p->update_ms += ms;
        p->updates += 1;
        p->gram_ms += ms;
        if (r.n_filled > 0) {
          p->gram_bytes += (double)r.n_occupied * (double)h->m * h->esize;
          p->gram_launches += 1;
          if (!h->gram_split) p->pool_copy_bytes += (double)r.n_filled * (double)h->m * h->esize;
        }
        if (h->gram_split && mk.aux >= 0) {
          // the split Gram copies, at the flush's last update, the basis
          // columns selected during the flush (column index >= its first)
          std::vector<int64_t> J(h->t);
          RID_HIP(h, hipMemcpy(J.data(), h->J_hist + (int64_t)mk.bytes * h->t, sizeof(int64_t) * h->t,
                               hipMemcpyDeviceToHost));
          int64_t nc = 0;
          for (int64_t j : J) nc += j >= mk.aux;
          p->pool_copy_bytes += (double)nc * (double)h->m * h->esize;
        }
        break;
      }
    }
  }
  return RID_OK;
}

static void destroy_stream(rid_stream* h) {
  if (h->side) (void)hipStreamSynchronize(h->side);
  (void)hipStreamSynchronize(h->s);
  (void)hipGetLastError();
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  free_all(h);
  delete h;
}

rid_status rid_destroy(rid_stream* h) {
  if (!h) return RID_EINVAL;
  if (h->owner) return fail(h, RID_ESTATE, "the stream belongs to a batch: use rid_destroy_batch");
  if (h->side) (void)hipStreamSynchronize(h->side);
  (void)hipStreamSynchronize(h->s);
  (void)hipGetLastError();
  free_all(h);
  delete h;
  return RID_OK;
}

rid_status rid_omega_block(int32_t prec, uint64_t omega_seed, int32_t ell, int64_t i0, int64_t count,
                           void* d_out, int64_t ld, void* stream) {
  if (prec < RID_SKETCH_F64 || prec > RID_SKETCH_FP8 || ell < 1 || ell > kMaxEll || i0 < 0 ||
      count < 0 || (count > 0 && !d_out) || ld < ell)
    return fail(nullptr, RID_EINVAL, "bad omega block arguments");
  if (count == 0) return RID_OK;
  hipError_t e = launch_omega_block(prec, omega_seed, ell, i0, count, d_out, ld,
                                    reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(nullptr, RID_EDEVICE, hipGetErrorString(e));
  return RID_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched streams.
//
// A batch owns ns member streams and an internal HIP stream on which all of
// their work runs.  A round advances every member by at most one lookahead
// batch: one persistent sketch launch walks the (stream, row slab, sketch
// rows, column tile) items of all members, one launch reduces them, and each
// update kernel runs once for all members with an update due (grid y = the
// member).  The argument tables of a round go to the device in one copy; the
// launches of a round are captured into a HIP graph whose executable is
// updated in place from round to round.  The row slab of the sketch is picked
// once per batch shape by timing the candidates on the first round's columns.
// ---------------------------------------------------------------------------
struct rid_batch {
  int ns = 0;
  uint32_t flags = 0;
  hipStream_t user = nullptr;  // the caller's stream
  hipStream_t s = nullptr;     // internal stream
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<rid_stream*> st;
  static constexpr int kSlots = 4;
  char* host_slot[kSlots] = {};
  hipEvent_t slot_ev[kSlots] = {};
  bool slot_used[kSlots] = {};
  int slot = 0;
  char* dev_tab = nullptr;
  size_t tab_cap = 0;
  hipGraphExec_t exec = nullptr;
  int64_t rounds = 0, graph_launches = 0, graph_instantiations = 0, graph_updates = 0;
  int64_t slab_rows = 0, min_slab_rows = 0;
  int wide = 0;  // bf16 members: the wide work split
  bool tuned = false;
  struct Cand {
    int64_t rows;
    int wide;
    double ms;
  };
  std::vector<Cand> tune_table;  // the timed candidates of the tuner
  double tune_ms = 0.0;
  int n_cu = 0;
  bool failed = false;
  std::string last_err;
  // timing (rounds then run as direct launches with events around each)
  bool profiling = false;
  struct Mark {
    hipEvent_t a, b;
    int kind;
    double bytes;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  int64_t prof_rounds = 0;
};

static hipEvent_t batch_event(rid_batch* bt) {
  if (!bt->event_pool.empty()) {
    hipEvent_t e = bt->event_pool.back();
    bt->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

static rid_status bfail(rid_batch* bt, rid_status st, const std::string& msg) {
  if (bt) {
    bt->last_err = msg;
    if (st == RID_EDEVICE || st == RID_ENUMERIC) {
      bt->failed = true;
      for (rid_stream* h : bt->st) fail(h, st, msg);
    }
  }
  g_last_err = msg;
  return st;
}

#define BT_HIP(bt, expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return bfail((bt), RID_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// slab candidates of the sketch (rows per work item)
static std::vector<int64_t> slab_candidates(int prec) {
  const int64_t cap = sketch_slab_cap(prec);
  std::vector<int64_t> v;
  for (int64_t r = 2048; r <= cap; r *= 2) v.push_back(r);
  return v;
}

static void set_slab(rid_stream* h, int64_t rows) {
  h->slab_rows = rows;
  h->n_slabs = (int)((h->m + rows - 1) / rows);
}

// Bytes of the argument tables of one round (upper bound).
static size_t table_bytes(int ns, int nzmax) {
  const size_t launches = 8 + (size_t)nzmax * 24;
  const size_t per_stream = 4 * sizeof(SketchArgs) + 4 * sizeof(BatchArgs) + 64 +
                            (size_t)nzmax * 24 * (sizeof(UpdArgs) + sizeof(int4));
  return (size_t)ns * per_stream + launches * 2 * 256 + (64 << 10);
}

// The next host staging slot (waits until the copy that last read it is done).
static rid_status take_slot(rid_batch* bt, Stage& stg) {
  bt->slot = (bt->slot + 1) % rid_batch::kSlots;
  if (bt->slot_used[bt->slot]) BT_HIP(bt, hipEventSynchronize(bt->slot_ev[bt->slot]));
  stg.host = bt->host_slot[bt->slot];
  stg.dev = bt->dev_tab;
  stg.cap = bt->tab_cap;
  stg.used = 0;
  stg.overflow = false;
  return RID_OK;
}

static rid_status copy_slot(rid_batch* bt, const Stage& stg) {
  if (stg.overflow) return bfail(bt, RID_EINVAL, "internal: argument tables exceed their staging buffer");
  if (stg.used) BT_HIP(bt, hipMemcpyAsync(bt->dev_tab, stg.host, stg.used, hipMemcpyHostToDevice, bt->s));
  BT_HIP(bt, hipEventRecord(bt->slot_ev[bt->slot], bt->s));
  bt->slot_used[bt->slot] = true;
  return RID_OK;
}

// Largest number of resident workgroups of a persistent sketch kernel.
static int sketch_grid_cap(rid_batch* bt, int prec) {
  return bt->n_cu * ((prec == RID_SKETCH_BF16 || prec == RID_SKETCH_FP8) ? 1 : 4);
}

static void plan_sketches(rid_batch* bt, const std::vector<SketchArgs>& args, const std::vector<int>& prec,
                          Stage& stg, std::vector<BLaunch>& out, bool with_reduce) {
  for (int p = RID_SKETCH_F64; p <= RID_SKETCH_FP8; ++p) {
    std::vector<SketchArgs> g;
    for (size_t i = 0; i < args.size(); ++i)
      if (prec[i] == p) g.push_back(args[i]);
    if (g.empty()) continue;
    plan_sketch_multi(p, g.data(), (int)g.size(), sketch_grid_cap(bt, p), stg, out);
    if (with_reduce) plan_sketch_reduce_b(p, g.data(), (int)g.size(), stg, out);
  }
}

// Runs the launches of a round: captured into the batch's graph (updated in
// place when the round has the same shape as the last one), or directly.
static rid_status batch_exec(rid_batch* bt, const std::vector<BLaunch>& L) {
  if (L.empty()) return RID_OK;
  if (bt->profiling) {
    for (const BLaunch& x : L) {
      rid_batch::Mark mk{batch_event(bt), batch_event(bt), x.kind, x.bytes};
      if (!mk.a || !mk.b) return bfail(bt, RID_EDEVICE, "event creation failed");
      BT_HIP(bt, hipEventRecord(mk.a, bt->s));
      BT_HIP(bt, run_launches(std::vector<BLaunch>{x}, bt->s));
      BT_HIP(bt, hipEventRecord(mk.b, bt->s));
      bt->marks.push_back(mk);
    }
    bt->prof_rounds += 1;
    return RID_OK;
  }
  if (bt->flags & RID_BATCH_NO_GRAPH) {
    BT_HIP(bt, run_launches(L, bt->s));
    return RID_OK;
  }
  hipGraph_t g = nullptr;
  BT_HIP(bt, hipStreamBeginCapture(bt->s, hipStreamCaptureModeThreadLocal));
  const hipError_t e1 = run_launches(L, bt->s);
  const hipError_t e2 = hipStreamEndCapture(bt->s, &g);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return bfail(bt, RID_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  if (bt->exec) {
    hipGraphNode_t en = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateSuccess;
    if (hipGraphExecUpdate(bt->exec, g, &en, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      bt->graph_updates += 1;
    } else {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(bt->exec);
      bt->exec = nullptr;
    }
  }
  if (!bt->exec) {
    const hipError_t e = hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      bt->exec = nullptr;
      (void)hipGraphDestroy(g);
      return bfail(bt, RID_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    bt->graph_instantiations += 1;
  }
  const hipError_t e = hipGraphLaunch(bt->exec, bt->s);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return bfail(bt, RID_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  bt->graph_launches += 1;
  return RID_OK;
}

// Picks the sketch slab of the batch by timing each candidate (sketch and
// reduction) on the columns of the first round (outside any graph); every
// candidate writes the same partial buffers, sketch columns and norms, which
// the real round overwrites afterwards.
static rid_status batch_tune(rid_batch* bt, const std::vector<int>& who, const std::vector<int64_t>& c0,
                             const std::vector<int>& b) {
  static std::vector<std::pair<std::string, int64_t>> cache;
  int64_t msum = 0;
  int prec = bt->st[0]->prec;
  for (rid_stream* h : bt->st) msum += h->m;
  char key[160];
  snprintf(key, sizeof(key), "p%d r%d ns%d m%lld b%d", prec, bt->st[0]->rbw, bt->ns,
           (long long)(msum >> 16), bt->st[0]->b_max);
  for (auto& kv : cache)
    if (kv.first == key) {
      bt->slab_rows = kv.second / 2;
      bt->wide = (int)(kv.second & 1);
      for (rid_stream* h : bt->st) {
        set_tile(h, h->cfg.sketch_tile == RID_TILE_WIDE || (h->cfg.sketch_tile == RID_TILE_AUTO && bt->wide));
        set_slab(h, bt->slab_rows);
      }
      bt->tuned = true;
      return RID_OK;
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BT_HIP(bt, hipEventCreate(&e0));
  BT_HIP(bt, hipEventCreate(&e1));
  double best = 1e300;
  int64_t best_rows = bt->slab_rows;
  int best_wide = 0;
  bool any_wide = false;
  // the wide split pads a round to 512-column tiles: a candidate only when
  // every lookahead batch fills at least two of them
  for (rid_stream* h : bt->st)
    any_wide = any_wide || (wide_applies(h) && h->cfg.sketch_tile == RID_TILE_AUTO && h->b_max >= 1024);
  // members that asked for a split keep it; the others take the candidate's
  auto apply_tile = [](rid_stream* h, int wide) {
    set_tile(h, h->cfg.sketch_tile == RID_TILE_WIDE || (h->cfg.sketch_tile == RID_TILE_AUTO && wide));
  };
  // Each candidate times the round's persistent sketch and reduction on one
  // column tile per member (the slab decides the per-item work, not how many
  // tiles there are): one untimed run, then the faster of two timed ones.
  // Candidates go by increasing slab; the times are U-shaped in the slab, so
  // the scan stops once a candidate runs 15% behind the best.
  for (int wide = 0; wide <= (any_wide ? 1 : 0); ++wide) {
  double best_here = 1e300;
  for (int64_t rows : slab_candidates(prec)) {
    if (rows < bt->min_slab_rows) continue;
    for (rid_stream* h : bt->st) {
      apply_tile(h, wide);
      set_slab(h, rows);
    }
    std::vector<SketchArgs> args;
    std::vector<int> precs;
    for (size_t i = 0; i < who.size(); ++i) {
      rid_stream* h = bt->st[who[i]];
      args.push_back(sketch_args(h, c0[i], std::min(b[i], h->cols_per_wg)));
      precs.push_back(h->prec);
    }
    float ms_rep[3] = {0.0f, 0.0f, 0.0f};
    for (int rep = 0; rep < 3; ++rep) {
      Stage stg;
      rid_status sts = take_slot(bt, stg);
      if (sts != RID_OK) return sts;
      std::vector<BLaunch> L;
      plan_sketches(bt, args, precs, stg, L, true);  // the reduction grows with the slab count
      if ((sts = copy_slot(bt, stg)) != RID_OK) return sts;
      BT_HIP(bt, hipEventRecord(e0, bt->s));
      BT_HIP(bt, run_launches(L, bt->s));
      BT_HIP(bt, hipEventRecord(e1, bt->s));
      BT_HIP(bt, hipEventSynchronize(e1));
      BT_HIP(bt, hipEventElapsedTime(&ms_rep[rep], e0, e1));
    }
    const float ms_last = std::min(ms_rep[1], ms_rep[2]);
    bt->tune_table.push_back(rid_batch::Cand{rows, wide, ms_last});
    bt->tune_ms += ms_rep[0] + ms_rep[1] + ms_rep[2];
    if (ms_last < best) {
      best = ms_last;
      best_rows = rows;
      best_wide = wide;
    }
    best_here = std::min(best_here, (double)ms_last);
    if (ms_last > 1.15 * best_here) break;
  }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  bt->slab_rows = best_rows;
  bt->wide = best_wide;
  for (rid_stream* h : bt->st) {
    apply_tile(h, best_wide);
    set_slab(h, best_rows);
  }
  cache.emplace_back(key, best_rows * 2 + best_wide);
  bt->tuned = true;
  return RID_OK;
}

enum RoundMode { ROUND_FULL = 0, ROUND_ALL = 1, ROUND_FINAL = 2 };

// One round; *worked is false when no member had anything to do.
static rid_status batch_round(rid_batch* bt, RoundMode mode, bool* worked) {
  *worked = false;
  const int ns = bt->ns;
  std::vector<int> sk_who, up_who;
  std::vector<int64_t> sk_c0;
  std::vector<int> sk_b, nfull(ns, 0), nlast(ns, 0), bsk(ns, 0);
  for (int i = 0; i < ns; ++i) {
    rid_stream* h = bt->st[i];
    if (h->finalized) continue;
    const int64_t pending = h->n_pushed - h->n_sketched;
    int b = 0;
    if (mode == ROUND_FULL) b = pending > h->b_max ? h->b_max : 0;
    else b = (int)std::min<int64_t>(h->b_max, pending);
    const int64_t nsk = h->n_sketched + b;
    // after the final partial update n_updates * t exceeds n_pushed: no more
    const int full = (int)std::max<int64_t>(0, nsk / h->t - h->n_updates);
    int last = 0;
    if (mode == ROUND_FINAL && nsk == h->n_pushed)
      last = (int)std::max<int64_t>(0, h->n_pushed - (h->n_updates + full) * h->t);
    bsk[i] = b;
    nfull[i] = full;
    nlast[i] = last;
    if (b > 0) {
      sk_who.push_back(i);
      sk_c0.push_back(h->n_sketched);
      sk_b.push_back(b);
    }
    if (full + (last > 0 ? 1 : 0) > 0) up_who.push_back(i);
  }
  if (sk_who.empty() && up_who.empty()) return RID_OK;
  *worked = true;
  rid_status sts;
  for (int i : sk_who)
    if ((sts = upload_colptrs(bt->st[i])) != RID_OK) return bfail(bt, RID_EDEVICE, bt->st[i]->last_err);
  if (!sk_who.empty() && !bt->tuned && !(bt->flags & RID_BATCH_NO_TUNE))
    if ((sts = batch_tune(bt, sk_who, sk_c0, sk_b)) != RID_OK) return sts;

  Stage stg;
  if ((sts = take_slot(bt, stg)) != RID_OK) return sts;
  std::vector<BLaunch> L;
  {
    std::vector<SketchArgs> args;
    std::vector<int> precs;
    for (size_t q = 0; q < sk_who.size(); ++q) {
      args.push_back(sketch_args(bt->st[sk_who[q]], sk_c0[q], sk_b[q]));
      precs.push_back(bt->st[sk_who[q]]->prec);
    }
    plan_sketches(bt, args, precs, stg, L, true);
  }
  int max_nz = 0;
  if (!up_who.empty()) {
    std::vector<BatchArgs> ba;
    for (int i : up_who) {
      rid_stream* h = bt->st[i];
      const int nz = nfull[i] + (nlast[i] > 0 ? 1 : 0);
      if (nz > h->nzmax) return bfail(bt, RID_EDEVICE, "internal: update batch larger than its slots");
      max_nz = std::max(max_nz, nz);
      ba.push_back(batch_args(h, nfull[i], nlast[i]));
    }
    plan_update_batch_b(ba.data(), (int)ba.size(), stg, L);
    {
      // Q of every update of the round depends on its tridiagonalisation only
      std::vector<UpdArgs> qa;
      for (int i : up_who)
        for (int z = 0; z < nfull[i] + (nlast[i] > 0 ? 1 : 0); ++z)
          qa.push_back(upd_args(bt->st[i], z, nfull[i], nlast[i]));
      plan_update_q_b(qa.data(), (int)qa.size(), stg, L);
    }
    // The coefficient phases of the round go last, in one launch per kernel
    // for every (member, update), against snapshots of each update's
    // selection state, when every member holds a buffer slice per update of
    // the round; else each step's phase follows its Gram.
    bool defer = true;
    for (int i : up_who)
      if (bt->st[i]->cgroup < nfull[i] + (nlast[i] > 0 ? 1 : 0)) defer = false;
    std::vector<UpdArgs> co;
    std::vector<char> co_p;   // the entry forms P (its member's last update of the round)
    for (int z = 0; z < max_nz; ++z) {
      std::vector<UpdArgs> ua;
      std::vector<char> ua_p;
      std::vector<SnapArgs> sa;
      for (int i : up_who) {
        rid_stream* h = bt->st[i];
        const int nz = nfull[i] + (nlast[i] > 0 ? 1 : 0);
        if (z >= nz) continue;
        UpdArgs a = upd_args(h, z, nfull[i], nlast[i]);
        a.flush_last = z == nz - 1;   // the member's last update of the round
        ua.push_back(a);
        ua_p.push_back(z == nz - 1);
        if (defer) {
          UpdArgs ac = a;
          ac.sc = h->sc_hist + a.u;
          ac.G = h->Ghist + (size_t)a.u * h->t * h->t;
          ac.J = h->J_hist + (size_t)a.u * h->t;
          coeff_slice(h, ac, z, nz);
          co.push_back(ac);
          co_p.push_back(z == nz - 1);
          sa.push_back(SnapArgs{a.sc, a.G, ac.sc, ac.G, h->t});
        }
      }
      plan_update_select_b(ua.data(), (int)ua.size(), stg, L, false);
      plan_update_gram_b(ua.data(), (int)ua.size(), stg, L);
      if (defer) {
        plan_update_snapshot_b(sa.data(), (int)sa.size(), stg, L);
      } else {
        std::unique_ptr<bool[]> wp(new bool[ua.size()]);
        for (size_t q = 0; q < ua.size(); ++q) wp[q] = ua_p[q] != 0;
        plan_update_coeff_b(ua.data(), (int)ua.size(), stg, L, wp.get());
      }
    }
    if (defer) {
      std::unique_ptr<bool[]> wp(new bool[co.size()]);
      for (size_t q = 0; q < co.size(); ++q) wp[q] = co_p[q] != 0;
      plan_update_coeff_b(co.data(), (int)co.size(), stg, L, wp.get());
    }
  }
  if ((sts = copy_slot(bt, stg)) != RID_OK) return sts;
  if ((sts = batch_exec(bt, L)) != RID_OK) return sts;
  for (int i = 0; i < ns; ++i) {
    rid_stream* h = bt->st[i];
    h->n_sketched += bsk[i];
    const int nz = nfull[i] + (nlast[i] > 0 ? 1 : 0);
    if (nz > 0) {
      h->sst_cur ^= 1;
      h->n_updates += nz;
      h->last_nobs = (h->n_updates - 1) * h->t + (nlast[i] > 0 ? nlast[i] : h->t);
    }
  }
  bt->rounds += 1;
  return RID_OK;
}

// COPY pushes: free ring space by sketching everything pending.
static rid_status batch_make_room(rid_batch* bt) {
  bool worked = true;
  while (worked) {
    rid_status st = batch_round(bt, ROUND_ALL, &worked);
    if (st != RID_OK) return st;
  }
  return RID_OK;
}

static rid_status batch_enter(rid_batch* bt) {
  BT_HIP(bt, hipEventRecord(bt->ev_in, bt->user));
  BT_HIP(bt, hipStreamWaitEvent(bt->s, bt->ev_in, 0));
  return RID_OK;
}

static rid_status batch_leave(rid_batch* bt) {
  BT_HIP(bt, hipEventRecord(bt->ev_out, bt->s));
  BT_HIP(bt, hipStreamWaitEvent(bt->user, bt->ev_out, 0));
  return RID_OK;
}

static void batch_free(rid_batch* bt) {
  if (bt->s) (void)hipStreamSynchronize(bt->s);
  (void)hipGetLastError();
  for (auto& mk : bt->marks) {
    (void)hipEventDestroy(mk.a);
    (void)hipEventDestroy(mk.b);
  }
  for (hipEvent_t e : bt->event_pool) (void)hipEventDestroy(e);
  for (rid_stream* h : bt->st) {
    h->owner = nullptr;
    destroy_stream(h);
  }
  bt->st.clear();
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  for (int i = 0; i < rid_batch::kSlots; ++i) {
    if (bt->host_slot[i]) (void)hipHostFree(bt->host_slot[i]);
    if (bt->slot_ev[i]) (void)hipEventDestroy(bt->slot_ev[i]);
  }
  if (bt->dev_tab) (void)hipFree(bt->dev_tab);
  if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
  if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
  if (bt->s) (void)hipStreamDestroy(bt->s);
  (void)hipGetLastError();
  delete bt;
}

extern "C" {

rid_status rid_init_batch(int32_t ns, const rid_config* cfgs, void* stream, uint32_t flags, rid_batch** out) {
  if (!cfgs || !out) return fail(nullptr, RID_EINVAL, "null argument");
  *out = nullptr;
  if (ns < 1 || ns > kMaxBatchStreams) return fail(nullptr, RID_EINVAL, "ns must be in [1, 4096]");
  if (flags & ~(RID_BATCH_NO_GRAPH | RID_BATCH_NO_TUNE)) return fail(nullptr, RID_EINVAL, "unknown batch flags");
  for (int i = 0; i < ns; ++i) {
    rid_status st = validate(&cfgs[i]);
    if (st != RID_OK) return st;
  }
  rid_batch* bt = new rid_batch();
  bt->ns = ns;
  bt->flags = flags;
  bt->user = reinterpret_cast<hipStream_t>(stream);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      hipStreamCreateWithFlags(&bt->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    batch_free(bt);
    return fail(nullptr, RID_EDEVICE, "batch stream or event creation failed");
  }
  bt->n_cu = prop.multiProcessorCount;
  int nzmax = 0;
  int64_t min_rows = 1 << 30;
  for (int i = 0; i < ns; ++i) {
    rid_stream* h = nullptr;
    rid_status st = init_stream(&cfgs[i], bt->s, &h, true);
    if (st != RID_OK) {
      const std::string msg = g_last_err;
      batch_free(bt);
      g_last_err = "member " + std::to_string(i) + ": " + msg;
      return st;
    }
    h->owner = bt;
    h->join = bt->user;
    bt->st.push_back(h);
    if (hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      batch_free(bt);
      return fail(nullptr, RID_EDEVICE, "event creation failed");
    }
    nzmax = std::max(nzmax, h->nzmax);
    min_rows = std::min(min_rows, slab_candidates(h->prec).front());
  }
  // every member keeps the slab geometry of the batch: partial buffers sized
  // for the smallest candidate, the default slab until the tuner has run
  bt->min_slab_rows = (flags & RID_BATCH_NO_TUNE) ? 16384 : min_rows;
  bt->slab_rows = 16384;
  for (rid_stream* h : bt->st) {
    const int64_t rows = std::min<int64_t>(bt->min_slab_rows, slab_candidates(h->prec).back());
    set_slab(h, rows);
    void* part = nullptr;
    double* normpart = nullptr;
    const size_t psize = (h->prec == RID_SKETCH_F64) ? 8 : 4;
    rid_status st = dalloc(h, &part, (size_t)h->n_slabs * h->b_max * h->ell_pad * psize);
    if (st == RID_OK) st = dalloc_t(h, &normpart, (size_t)h->n_slabs * h->b_max);
    if (st != RID_OK) {
      batch_free(bt);
      return st;
    }
    dfree(h, h->part);
    dfree(h, h->normpart);
    h->part = part;
    h->normpart = normpart;
    set_slab(h, std::min<int64_t>(bt->slab_rows, slab_candidates(h->prec).back()));
  }
  bt->tab_cap = table_bytes(ns, nzmax);
  if (hipMalloc(reinterpret_cast<void**>(&bt->dev_tab), bt->tab_cap) != hipSuccess) {
    (void)hipGetLastError();
    batch_free(bt);
    return fail(nullptr, RID_ENOMEM, "argument table allocation failed");
  }
  for (int i = 0; i < rid_batch::kSlots; ++i)
    if (hipHostMalloc(reinterpret_cast<void**>(&bt->host_slot[i]), bt->tab_cap, hipHostMallocDefault) !=
            hipSuccess ||
        hipEventCreateWithFlags(&bt->slot_ev[i], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      batch_free(bt);
      return fail(nullptr, RID_ENOMEM, "staging allocation failed");
    }
  *out = bt;
  return RID_OK;
}

rid_status rid_push_batch(rid_batch* bt, const void* const* d_cols, const int64_t* ld, const int32_t* b,
                          uint32_t flags) {
  if (!bt) return fail(nullptr, RID_EINVAL, "null batch");
  if (bt->failed) return bfail(bt, RID_ESTATE, "batch failed");
  if (!d_cols || !ld || !b) return bfail(bt, RID_EINVAL, "null argument");
  if (flags != RID_COPY && flags != RID_BORROW) return bfail(bt, RID_EINVAL, "bad flags");
  for (int i = 0; i < bt->ns; ++i) {
    rid_stream* h = bt->st[i];
    if (b[i] < 0 || (b[i] > 0 && (!d_cols[i] || ld[i] < h->m))) return bfail(bt, RID_EINVAL, "bad push arguments");
    if (b[i] > 0 && h->finalized) return bfail(bt, RID_ESTATE, "stream finalized");
    if (h->n_pushed + b[i] > h->n_max) return bfail(bt, RID_ECAPACITY, "push exceeds n_max");
    if (flags == RID_BORROW && b[i] > 0 &&
        (reinterpret_cast<uintptr_t>(d_cols[i]) % 16 != 0 || (ld[i] * h->esize) % 16 != 0))
      return bfail(bt, RID_EINVAL, "BORROW needs 16-byte aligned columns (pointer and ld * size)");
  }
  rid_status st = batch_enter(bt);
  if (st != RID_OK) return st;
  for (int i = 0; i < bt->ns; ++i)
    if (b[i] > 0 && (st = push_columns(bt->st[i], d_cols[i], ld[i], b[i], flags, false)) != RID_OK)
      return bfail(bt, st == RID_EDEVICE ? RID_EDEVICE : st, bt->st[i]->last_err);
  bool worked = true;
  while (worked)
    if ((st = batch_round(bt, ROUND_FULL, &worked)) != RID_OK) return st;
  return batch_leave(bt);
}

rid_status rid_finalize_batch(rid_batch* bt) {
  if (!bt) return fail(nullptr, RID_EINVAL, "null batch");
  if (bt->failed) return bfail(bt, RID_ESTATE, "batch failed");
  rid_status st = batch_enter(bt);
  if (st != RID_OK) return st;
  bool worked = true;
  while (worked)
    if ((st = batch_round(bt, ROUND_FINAL, &worked)) != RID_OK) return st;
  for (rid_stream* h : bt->st) h->finalized = true;
  return batch_leave(bt);
}

rid_status rid_batch_stream(rid_batch* bt, int32_t i, rid_stream** out) {
  if (!bt || !out) return fail(nullptr, RID_EINVAL, "null argument");
  if (i < 0 || i >= bt->ns) return bfail(bt, RID_EINVAL, "member index out of range");
  *out = bt->st[i];
  return RID_OK;
}

rid_status rid_batch_get_info(rid_batch* bt, rid_batch_info* info) {
  if (!bt || !info) return fail(nullptr, RID_EINVAL, "null argument");
  if (!bt->failed) {
    hipError_t e = hipStreamSynchronize(bt->s);
    if (e != hipSuccess) bfail(bt, RID_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  }
  memset(info, 0, sizeof(*info));
  info->ns = bt->ns;
  info->failed = bt->failed ? 1 : 0;
  info->rounds = bt->rounds;
  info->graph_launches = bt->graph_launches;
  info->graph_instantiations = bt->graph_instantiations;
  info->graph_updates = bt->graph_updates;
  info->slab_rows = bt->slab_rows;
  info->tuned = bt->tuned ? 1 : 0;
  info->wide = 0;
  for (rid_stream* h : bt->st) info->wide |= h->wide;
  info->tune_ms = bt->tune_ms;
  return RID_OK;
}

rid_status rid_batch_tune_result(rid_batch* bt, int32_t i, int64_t* slab_rows, int32_t* wide, double* ms) {
  if (!bt || !slab_rows || !wide || !ms) return fail(nullptr, RID_EINVAL, "null argument");
  if (i < 0 || i >= (int32_t)bt->tune_table.size()) return RID_EINVAL;
  *slab_rows = bt->tune_table[i].rows;
  *wide = bt->tune_table[i].wide;
  *ms = bt->tune_table[i].ms;
  return RID_OK;
}

rid_status rid_batch_last_error(rid_batch* bt, char* buf, size_t n) {
  if (!buf || n == 0) return RID_EINVAL;
  snprintf(buf, n, "%s", bt ? bt->last_err.c_str() : g_last_err.c_str());
  return RID_OK;
}

rid_status rid_reset_batch(rid_batch* bt) {
  if (!bt) return fail(nullptr, RID_EINVAL, "null batch");
  if (bt->failed) return bfail(bt, RID_ESTATE, "batch failed");
  rid_status st = batch_enter(bt);
  if (st != RID_OK) return st;
  for (rid_stream* h : bt->st)
    if ((st = reset_stream(h)) != RID_OK) return bfail(bt, st, h->last_err);
  return batch_leave(bt);
}

rid_status rid_batch_profile_enable(rid_batch* bt, int32_t on) {
  if (!bt) return fail(nullptr, RID_EINVAL, "null batch");
  BT_HIP(bt, hipStreamSynchronize(bt->s));
  for (auto& mk : bt->marks) {
    bt->event_pool.push_back(mk.a);
    bt->event_pool.push_back(mk.b);
  }
  bt->marks.clear();
  bt->prof_rounds = 0;
  bt->profiling = on != 0;
  return RID_OK;
}

rid_status rid_batch_profile_read(rid_batch* bt, rid_profile* p) {
  if (!bt || !p) return fail(nullptr, RID_EINVAL, "null argument");
  BT_HIP(bt, hipStreamSynchronize(bt->s));
  memset(p, 0, sizeof(*p));
  for (auto& mk : bt->marks) {
    float ms = 0.0f;
    BT_HIP(bt, hipEventElapsedTime(&ms, mk.a, mk.b));
    switch (mk.kind) {
      case 0: p->sketch_ms += ms; p->sketch_launches += 1; p->sketch_bytes += mk.bytes; break;
      case 1: p->reduce_ms += ms; break;
      case 3: p->gram_ms += ms; p->update_ms += ms; break;
      default: p->update_ms += ms; break;
    }
  }
  p->updates = bt->prof_rounds;
  return RID_OK;
}

rid_status rid_destroy_batch(rid_batch* bt) {
  if (!bt) return RID_EINVAL;
  batch_free(bt);
  return RID_OK;
}

}  // extern "C"
