// Host runtime and C ABI: plans, batches, launch schedules, HIP-graph replay.
//
// A batch owns, per configuration, two front pools (the frontal Gauss-Jordan sweep
// ping-pongs between them; the selected-inverse front of a supernode lands in the
// pool its factorised front does not occupy), a complex and an int workspace, the
// links, their inverses and the gathered selected blocks. All launch descriptors
// are built once at batch creation from the immutable plan; a numeric call only
// walks the precomputed launch list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/clsel.h"
#include "desc.hpp"
#include "kernels.hpp"
#include "layout.hpp"
#include "plan.hpp"

using clsel::Launch;
using clsel::Layout;
using clsel::SolveLayout;
using clsel::cdiv64;
using clsel::build_layout;
using clsel::validate_layout;
using clsel::layout_bytes;
using clsel::build_solve_layout;
using clsel::validate_solve_layout;
using clsel::kAsm;
using clsel::kPanel;
using clsel::kGemm;
using clsel::kZss;
using clsel::kRhsAsm;
using clsel::kRhsGather;
using clsel::kSolScatter;

struct cl_plan_s {
  clsel::Plan P;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(CL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

struct cl_batch_s {
  cl_plan plan = nullptr;
  Layout L;
  int cap = 0, active = 0;
  int device = 0;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_param = nullptr;
  // cl_run in two lanes: the second half of the configurations on a second stream
  // (forked from and joined back to st), so that the latency-bound kernels of one half
  // (pivot panels, assembly, gathers) run beside the other half's GEMMs
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int lanes = 0;  // 0: two lanes from kAutoLaneBatch active configurations, else 1 or 2
  double2* fronts = nullptr;
  double2* ws = nullptr;
  int32_t* iws = nullptr;
  double2* links = nullptr;
  double2* linv = nullptr;
  double2* sel = nullptr;
  double* params = nullptr;       // device: m[cap], mu[cap]
  double* lparams = nullptr;      // device: beta[cap], eps_bar[cap], kref[cap] (Langevin step)
  double* lparams_host = nullptr; // pinned staging of lparams
  hipEvent_t ev_lparam = nullptr; // the last lparams upload has left the pinned buffer
  unsigned long long* kmax = nullptr;  // device [cap]: max_link |K| as a bit pattern
  // multi-RHS solves: layout for the last n, its descriptors and the workspace
  SolveLayout solve;
  char* solve_blob = nullptr;
  double2* rhs = nullptr;
  // the low-rank correction's right and left solves (R right-hand sides), their shared
  // workspace, and the global index of every pivot column
  SolveLayout smw_r, smw_l;
  char* smw_blob_r = nullptr;
  char* smw_blob_l = nullptr;
  double2* smw_rhs = nullptr;
  int32_t* d_pivglob = nullptr;
  double* params_host = nullptr;  // pinned staging
  int32_t* status = nullptr;
  char* dblob = nullptr;
  int32_t* d_front_sites = nullptr;
  int32_t* d_site_coords = nullptr;
  int32_t* d_inv = nullptr;
  int32_t* d_rel = nullptr;
  int64_t* d_sel_off = nullptr;
  int32_t* d_sel_ld = nullptr;
  int state = 0;  // 0 created, 1 factored, 2 inverted
  int fault_cfg = -1, fault_front = -1;  // test support: a zeroed pivot block
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  int g_lanes = 0;
  const void* g_links = nullptr;
  void* g_sel = nullptr;
  void* g_drift = nullptr;
  int g_active = 0;
  // optional per-launch timing of the GEMM kernels (HIP events on the batch stream)
  int prof = 0;                      // bit k set: time GEMM launches of mode k
  std::vector<hipEvent_t> prof_ev;   // pairs, recorded around each GEMM launch
  std::vector<double> prof_flops;    // algorithmic flops of each timed launch
  std::vector<double> prof_bytes;    // algorithmic bytes of each timed launch
  std::vector<int32_t> prof_mode;    // GEMM mode of each timed launch
  size_t prof_used = 0;
  double prof_ms = 0, prof_flop_total = 0, prof_byte_total = 0;
  int64_t prof_launches = 0;
};

namespace {

template <class T>
int dalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? CL_ENOMEM : CL_EHIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return 0;
}

template <class T>
int upload(T** p, const std::vector<T>& v) {
  int rc = dalloc(p, v.size());
  if (rc) return rc;
  if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return 0;
}

clsel::LatticeDims ldims(const clsel::Plan& P) {
  clsel::LatticeDims d;
  for (int k = 0; k < 4; ++k) d.L[k] = P.dims[k];
  return d;
}

int enqueue_launches(cl_batch b, const std::vector<Launch>& ls) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  for (const Launch& l : ls) {
    if (l.gridx <= 0) continue;
    const dim3 grid((unsigned)l.gridx, (unsigned)B);
    const char* dp = b->dblob + l.desc_off;
    switch (l.kind) {
      case kAsm:
        hipLaunchKernelGGL(clsel::k_assemble, grid, dim3(256), 0, b->st,
                           (const clsel::AsmDesc*)dp, l.count, b->fronts, b->L.cfg_stride,
                           b->d_front_sites, b->d_inv, (const uint32_t*)b->d_site_coords, b->links,
                           b->linv, b->L.links_elems,
                           b->params, b->params + b->cap, ldims(P), b->iws, b->L.iws_elems,
                           b->fault_cfg, b->fault_front);
        break;
      case kPanel:
        clsel::launch_panel(l.rpt, grid, b->st, (const clsel::PanelDesc*)dp, b->fronts,
                            b->L.cfg_stride, b->ws, b->L.ws_elems, b->iws, b->L.iws_elems,
                            b->status, b->L.R > 0 ? P.opt.pivot_floor : 0.0);
        break;
      case kGemm: {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool timed = (b->prof >> l.rpt) & 1;
        if (timed) {
          if (b->prof_used + 2 > b->prof_ev.size()) {
            for (int k = 0; k < 64; ++k) {
              hipEvent_t e;
              HIPCHK(hipEventCreate(&e));
              b->prof_ev.push_back(e);
            }
          }
          e0 = b->prof_ev[b->prof_used];
          e1 = b->prof_ev[b->prof_used + 1];
          b->prof_used += 2;
          b->prof_flops.push_back(l.flops * B);
          b->prof_bytes.push_back(l.bytes * B);
          b->prof_mode.push_back(l.rpt);
          HIPCHK(hipEventRecord(e0, b->st));
        }
        clsel::launch_gemm(l.rpt, l.tile, grid, b->st, (const clsel::GemmDesc*)dp, l.count, b->fronts,
                           b->L.cfg_stride, P.pool_elems, b->ws, b->L.ws_elems, b->iws,
                           b->L.iws_elems, nullptr, 0, b->d_inv);
        if (timed) HIPCHK(hipEventRecord(e1, b->st));
        break;
      }
      case kZss:
        hipLaunchKernelGGL(clsel::k_gather_zss, grid, dim3(256), 0, b->st,
                           (const clsel::GatherDesc*)dp, l.count, b->fronts, b->L.cfg_stride,
                           b->d_rel);
        break;
    }
    HIPCHK(hipGetLastError());
  }
  return 0;
}

int enqueue_smw(cl_batch b);
clsel::SmwCtx smw_ctx(cl_batch b);

int upload_params(cl_batch b, bool capturing) {
  HIPCHK(hipMemcpyAsync(b->params, b->params_host, sizeof(double) * 2 * b->cap,
                        hipMemcpyHostToDevice, b->st));
  // marks the pinned staging buffer reusable; under capture it is recorded after the launch
  if (!capturing) HIPCHK(hipEventRecord(b->ev_param, b->st));
  return 0;
}

// The factorisation of the active configurations; m and mu are already on the device.
int enqueue_factor_body(cl_batch b, const void* links_dev) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  HIPCHK(hipMemcpyAsync(b->links, links_dev, sizeof(double2) * b->L.links_elems * B,
                        hipMemcpyDeviceToDevice, b->st));
  hipLaunchKernelGGL(k_fill_i32, dim3((B + 255) / 256), dim3(256), 0, b->st, b->status, B, 0);
  HIPCHK(hipGetLastError());
  const int64_t nl = P.V * 4 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_link_inverse, dim3((unsigned)cdiv64(nl, 256)), dim3(256), 0, b->st,
                     b->links, b->linv, P.V * 4, B, b->status);
  HIPCHK(hipGetLastError());
  int rc = enqueue_launches(b, b->L.factor);
  if (rc || b->L.R == 0) return rc;
  // the perturbed pivots of each configuration, in pivot-column order (CL_ERANK past the cap)
  hipLaunchKernelGGL(clsel::k_smw_list, dim3(B), dim3(256), 0, b->st, smw_ctx(b));
  HIPCHK(hipGetLastError());
  return 0;
}

int enqueue_factor(cl_batch b, const void* links_dev, bool capturing) {
  int rc = upload_params(b, capturing);
  return rc ? rc : enqueue_factor_body(b, links_dev);
}

int enqueue_selinv(cl_batch b) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  int rc = enqueue_launches(b, b->L.selinv);
  if (rc) return rc;
  const int64_t n = P.V * 81 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_gather_selected, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0,
                     b->st, b->fronts, b->L.cfg_stride, b->d_sel_off, b->d_sel_ld, P.V, B,
                     b->status, b->sel);
  HIPCHK(hipGetLastError());
  return enqueue_smw(b);
}

int enqueue_selected(cl_batch b, void* out) {
  HIPCHK(hipMemcpyAsync(out, b->sel, sizeof(double2) * b->L.sel_elems * b->active,
                        hipMemcpyDeviceToDevice, b->st));
  return 0;
}

int enqueue_drift(cl_batch b, void* out) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  const int64_t n = P.V * 4 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_drift, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, b->st, b->sel,
                     b->links, b->linv, b->params + b->cap, ldims(P), P.V, B, (double2*)out);
  HIPCHK(hipGetLastError());
  return 0;
}

// Configurations [b0, b0 + n) of the batch as a batch of n on stream st, for the scope of
// this object: every per-configuration buffer pointer moves to configuration b0 (the
// kernels address configuration blockIdx.y from those pointers and their per-configuration
// strides) and is put back at the end. Host-side only; a batch is not used concurrently.
class SubBatch {
 public:
  SubBatch(cl_batch b, int b0, int n, hipStream_t st) : b_(b), s_(*b) {
    const Layout& L = b->L;
    b->fronts += b0 * L.cfg_stride;
    b->ws += b0 * L.ws_elems;
    b->iws += b0 * L.iws_elems;
    b->links += b0 * L.links_elems;
    b->linv += b0 * L.links_elems;
    b->sel += b0 * L.sel_elems;
    b->params += b0;  // m at [0, cap), mu at [cap, 2 cap): both move by b0
    b->lparams += b0;
    b->kmax += b0;
    b->status += b0;
    if (b->rhs) b->rhs += b0 * b->solve.stride;
    if (b->smw_rhs) b->smw_rhs += b0 * std::max(b->smw_r.stride, b->smw_l.stride);
    b->fault_cfg = (b->fault_cfg >= b0 && b->fault_cfg < b0 + n) ? b->fault_cfg - b0 : -1;
    b->active = n;
    b->st = st;
  }
  ~SubBatch() { s_.put(b_); }
  SubBatch(const SubBatch&) = delete;
  SubBatch& operator=(const SubBatch&) = delete;

 private:
  struct Saved {
    double2 *fronts, *ws, *links, *linv, *sel, *rhs, *smw_rhs;
    int32_t *iws, *status;
    double *params, *lparams;
    unsigned long long* kmax;
    int active, fault_cfg;
    hipStream_t st;
    explicit Saved(const cl_batch_s& b)
        : fronts(b.fronts), ws(b.ws), links(b.links), linv(b.linv), sel(b.sel), rhs(b.rhs),
          smw_rhs(b.smw_rhs), iws(b.iws), status(b.status), params(b.params), lparams(b.lparams),
          kmax(b.kmax), active(b.active), fault_cfg(b.fault_cfg), st(b.st) {}
    void put(cl_batch b) const {
      b->fronts = fronts; b->ws = ws; b->links = links; b->linv = linv; b->sel = sel; b->rhs = rhs;
      b->smw_rhs = smw_rhs; b->iws = iws; b->status = status; b->params = params;
      b->lparams = lparams; b->kmax = kmax; b->active = active; b->fault_cfg = fault_cfg; b->st = st;
    }
  };
  cl_batch b_;
  Saved s_;
};

// Lanes cl_run uses for the active configurations: two from this many on (each half keeps
// enough configurations to fill the device in its GEMM launches), unless set explicitly;
// one while GEMM launches are being timed.
constexpr int kAutoLaneBatch = 16;
int run_lanes(cl_batch b) {
  if (b->prof || b->active < 2) return 1;
  if (b->lanes) return b->lanes;
  return b->active >= kAutoLaneBatch ? 2 : 1;
}

// cl_run's work: factorisation, selected inversion with the low-rank correction,
// selected blocks and drift of the active configurations, in one or two lanes.
int enqueue_run(cl_batch b, const void* links_dev, void* sel_out, void* drift_out, bool capturing) {
  int rc = upload_params(b, capturing);
  if (rc) return rc;
  auto body = [&](const void* lk, void* so, void* dr) -> int {
    int r = enqueue_factor_body(b, lk);
    if (!r) r = enqueue_selinv(b);
    if (!r && so) r = enqueue_selected(b, so);
    if (!r && dr) r = enqueue_drift(b, dr);
    return r;
  };
  const int nl = run_lanes(b);
  if (nl == 1) return body(links_dev, sel_out, drift_out);
  const clsel::Plan& P = b->plan->P;
  const int B = b->active, h = B / 2;
  HIPCHK(hipEventRecord(b->ev_fork, b->st));
  HIPCHK(hipStreamWaitEvent(b->st2, b->ev_fork, 0));
  for (int lane = 0; lane < 2 && !rc; ++lane) {
    const int b0 = lane ? h : 0, n = lane ? B - h : h;
    SubBatch sb(b, b0, n, lane ? b->st2 : b->st);
    rc = body((const double2*)links_dev + b0 * b->L.links_elems,
              sel_out ? (void*)((double2*)sel_out + b0 * b->L.sel_elems) : nullptr,
              drift_out ? (void*)((double2*)drift_out + b0 * P.V * 32) : nullptr);
  }
  // the join is recorded even after an error, so that a capture still ends on st
  HIPCHK(hipEventRecord(b->ev_join, b->st2));
  HIPCHK(hipStreamWaitEvent(b->st, b->ev_join, 0));
  return rc;
}

int begin(cl_batch b) {
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipEventRecord(b->ev_in, b->user));
  HIPCHK(hipStreamWaitEvent(b->st, b->ev_in, 0));
  return 0;
}

int end(cl_batch b) {
  HIPCHK(hipEventRecord(b->ev_out, b->st));
  HIPCHK(hipStreamWaitEvent(b->user, b->ev_out, 0));
  return 0;
}

int stage_params(cl_batch b, const double* m, const double* mu) {
  // the previous call's parameter upload must have left the pinned buffer
  HIPCHK(hipEventSynchronize(b->ev_param));
  for (int i = 0; i < b->active; ++i) {
    b->params_host[i] = m[i];
    b->params_host[b->cap + i] = mu[i];
  }
  return 0;
}

void free_batch(cl_batch b) {
  if (!b) return;
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  hipFree(b->fronts); hipFree(b->ws); hipFree(b->iws); hipFree(b->links); hipFree(b->linv);
  hipFree(b->sel); hipFree(b->params); hipFree(b->status); hipFree(b->dblob);
  hipFree(b->lparams); hipFree(b->kmax);
  hipFree(b->solve_blob); hipFree(b->rhs);
  hipFree(b->smw_blob_r); hipFree(b->smw_blob_l); hipFree(b->smw_rhs); hipFree(b->d_pivglob);
  if (b->lparams_host) hipHostFree(b->lparams_host);
  if (b->ev_lparam) hipEventDestroy(b->ev_lparam);
  hipFree(b->d_front_sites); hipFree(b->d_site_coords); hipFree(b->d_inv); hipFree(b->d_rel); hipFree(b->d_sel_off);
  hipFree(b->d_sel_ld);
  if (b->params_host) hipHostFree(b->params_host);
  for (hipEvent_t e : b->prof_ev) hipEventDestroy(e);
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->ev_param) hipEventDestroy(b->ev_param);
  if (b->ev_fork) hipEventDestroy(b->ev_fork);
  if (b->ev_join) hipEventDestroy(b->ev_join);
  if (b->st2) hipStreamDestroy(b->st2);
  if (b->st) hipStreamDestroy(b->st);
  delete b;
}

}  // namespace

extern "C" {

const char* cl_strerror(int code) {
  switch (code) {
    case CL_OK: return "ok";
    case CL_EINVAL: return "invalid argument";
    case CL_ENOMEM: return "out of memory";
    case CL_EORDER: return "call out of order";
    case CL_ESINGULAR: return "singular pivot block";
    case CL_ENONFINITE: return "non-finite or singular link";
    case CL_EHIP: return "HIP runtime error";
    case CL_ENODEV: return "no usable GPU";
    case CL_ERANK: return "more perturbed pivots than the low-rank correction holds";
    default: return "unknown error";
  }
}

const char* cl_last_error(void) { return g_err.c_str(); }

int cl_symbolic_ex(const int32_t dims[4], const cl_plan_opts* opts, cl_plan* out) {
  if (!dims || !out) return fail(CL_EINVAL, "null pointer");
  clsel::PlanOptions o;
  if (opts) {
    if (opts->leaf_sites > 0) o.leaf_sites = opts->leaf_sites;
    if (opts->max_pivot_rows > 0) o.max_pivot_rows = opts->max_pivot_rows;
    if (opts->nb > 0) o.nb = opts->nb;
    o.time_cuts = opts->time_cuts != 0;
    o.gemm_tile = opts->gemm_tile;
    if (opts->lowrank_cap != 0) o.lowrank_cap = opts->lowrank_cap;
    if (opts->pivot_floor != 0.0) o.pivot_floor = opts->pivot_floor;
    o.smw_refine = opts->smw_refine;
  }
  if (o.gemm_tile != 0 && o.gemm_tile != clsel::kTile64 && o.gemm_tile != clsel::kTile128x64 &&
      o.gemm_tile != clsel::kTile128)
    return fail(CL_EINVAL, "gemm_tile must be 0, 64, 12864 or 128");
  if (o.max_pivot_rows > clsel::kMaxPivotRows || o.max_pivot_rows < 3)
    return fail(CL_EINVAL, "max_pivot_rows must be in [3, 1536]");
  if (o.nb > clsel::kMaxNB) return fail(CL_EINVAL, "nb must be in [1, 64]");
  cl_plan p = new (std::nothrow) cl_plan_s;
  if (!p) return fail(CL_ENOMEM, "plan allocation");
  std::string err;
  if (clsel::build_plan(dims, o, p->P, err) != 0) {
    delete p;
    return fail(CL_EINVAL, err);
  }
  *out = p;
  return 0;
}

int cl_symbolic(const int32_t dims[4], cl_plan* out) { return cl_symbolic_ex(dims, nullptr, out); }

int cl_plan_info(cl_plan plan, cl_plan_info_t* o) {
  if (!plan || !o) return fail(CL_EINVAL, "null pointer");
  const clsel::Plan& P = plan->P;
  for (int k = 0; k < 4; ++k) o->dims[k] = P.dims[k];
  o->volume = P.V;
  o->n = P.N;
  o->nfronts = (int32_t)P.fronts.size();
  o->nlevels = (int32_t)P.levels.size();
  o->max_steps = P.max_steps;
  o->max_front_rows = P.max_H;
  o->max_pivot_rows = P.max_p;
  o->pool_elems = P.pool_elems;
  o->flops_factor = P.flops_factor_exec;
  o->flops_selinv = P.flops_selinv_exec;
  o->flops_factor_alg = P.flops_factor_alg;
  o->flops_selinv_alg = P.flops_selinv_alg;
  o->flops_dense_inverse = P.flops_dense_inverse;
  o->lowrank_cap = P.opt.lowrank_cap;
  o->pivot_floor = P.opt.pivot_floor;
  o->smw_refine = P.opt.smw_refine;
  return 0;
}

size_t cl_plan_bytes(cl_plan plan, int32_t batch) {
  if (!plan || batch < 1) return 0;
  Layout L;
  build_layout(plan->P, L);
  std::string why;
  if (!validate_layout(plan->P, L, why)) { g_err = why; return 0; }
  return layout_bytes(plan->P, L, batch);
}

int cl_plan_export(cl_plan plan, int32_t what, void* dst, size_t* nbytes) {
  if (!plan || !nbytes) return fail(CL_EINVAL, "null pointer");
  const clsel::Plan& P = plan->P;
  std::vector<int64_t> rows;
  const void* src = nullptr;
  size_t n = 0;
  switch (what) {
    case 0:
      for (const clsel::Front& f : P.fronts) {
        const int64_t r[CL_FRONT_FIELDS] = {
            f.id, f.parent, f.level, f.npiv, f.nstr, f.p, f.s, f.H, f.ld, f.off, f.site_off,
            f.nchild, f.child[0], f.child[1], f.child[2], f.child[3], f.inv_off[0], f.inv_off[1],
            f.inv_off[2], f.inv_off[3], f.rel_off, f.nsteps, f.fbuf, f.zbuf, 0, 0, 0, 0};
        rows.insert(rows.end(), r, r + CL_FRONT_FIELDS);
      }
      src = rows.data(); n = rows.size() * 8; break;
    case 1: src = P.front_sites.data(); n = P.front_sites.size() * 4; break;
    case 2: src = P.inv_maps.data(); n = P.inv_maps.size() * 4; break;
    case 3: src = P.rel_maps.data(); n = P.rel_maps.size() * 4; break;
    case 4: src = P.sel_off.data(); n = P.sel_off.size() * 8; break;
    case 5: src = P.order.data(); n = P.order.size() * 8; break;
    default: return fail(CL_EINVAL, "unknown table");
  }
  if (dst) {
    if (*nbytes < n) return fail(CL_EINVAL, "destination too small");
    std::memcpy(dst, src, n);
  }
  *nbytes = n;
  return 0;
}

void cl_plan_destroy(cl_plan plan) { delete plan; }

int cl_batch_create(cl_plan plan, int32_t batch, void* hip_stream, cl_batch* out) {
  if (!plan || !out || batch < 1 || batch > 65535) return fail(CL_EINVAL, "bad plan, batch or output");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(CL_ENODEV, "no GPU visible");
  cl_batch b = new (std::nothrow) cl_batch_s;
  if (!b) return fail(CL_ENOMEM, "batch allocation");
  b->plan = plan;
  b->cap = b->active = batch;
  b->user = (hipStream_t)hip_stream;
  const clsel::Plan& P = plan->P;
  build_layout(P, b->L);
  {
    std::string why;
    if (!validate_layout(P, b->L, why)) { delete b; return fail(CL_EINVAL, "launch table check failed: " + why); }
  }
  int rc = 0;
#define TRY(x) do { rc = (x); if (rc) { free_batch(b); return rc; } } while (0)
#define HTRY(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { free_batch(b); return fail(CL_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); } } while (0)
  HTRY(hipGetDevice(&b->device));
  HTRY(hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking));
  HTRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
  HTRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
  HTRY(hipEventCreateWithFlags(&b->ev_param, hipEventDisableTiming));
  HTRY(hipEventRecord(b->ev_param, b->st));
  HTRY(hipStreamCreateWithFlags(&b->st2, hipStreamNonBlocking));
  HTRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
  HTRY(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
  const int64_t B = batch;
  TRY(dalloc(&b->fronts, (size_t)(B * b->L.cfg_stride)));
  TRY(dalloc(&b->ws, (size_t)(B * b->L.ws_elems)));
  TRY(dalloc(&b->iws, (size_t)(B * b->L.iws_elems)));
  TRY(dalloc(&b->links, (size_t)(B * b->L.links_elems)));
  TRY(dalloc(&b->linv, (size_t)(B * b->L.links_elems)));
  TRY(dalloc(&b->sel, (size_t)(B * b->L.sel_elems)));
  TRY(dalloc(&b->params, (size_t)(2 * B)));
  TRY(dalloc(&b->lparams, (size_t)(3 * B)));
  TRY(dalloc(&b->kmax, (size_t)B));
  {
    hipError_t e = hipHostMalloc((void**)&b->lparams_host, sizeof(double) * 3 * B, hipHostMallocDefault);
    if (e != hipSuccess) { b->lparams_host = nullptr; free_batch(b); return fail(CL_ENOMEM, "pinned staging"); }
    std::memset(b->lparams_host, 0, sizeof(double) * 3 * B);
  }
  HTRY(hipEventCreateWithFlags(&b->ev_lparam, hipEventDisableTiming));
  HTRY(hipEventRecord(b->ev_lparam, b->st));
  TRY(dalloc(&b->status, (size_t)B));
  {
    hipError_t e = hipHostMalloc((void**)&b->params_host, sizeof(double) * 2 * B, hipHostMallocDefault);
    if (e != hipSuccess) { b->params_host = nullptr; free_batch(b); return fail(CL_ENOMEM, "pinned staging"); }
    std::memset(b->params_host, 0, sizeof(double) * 2 * B);
  }
  TRY(dalloc(&b->dblob, b->L.blob.size()));
  HTRY(hipMemcpy(b->dblob, b->L.blob.data(), b->L.blob.size(), hipMemcpyHostToDevice));
  TRY(upload(&b->d_front_sites, P.front_sites));
  TRY(upload(&b->d_site_coords, P.site_coords));
  TRY(upload(&b->d_inv, P.inv_maps));
  TRY(upload(&b->d_rel, P.rel_maps));
  TRY(upload(&b->d_sel_off, P.sel_off));
  TRY(upload(&b->d_sel_ld, P.sel_ld));
  if (b->L.R > 0) {  // the correction's right and left solves, R right-hand sides each
    std::string why;
    build_solve_layout(P, b->L, b->L.R, false, 0, b->smw_r, true);
    build_solve_layout(P, b->L, b->L.R, true, 0, b->smw_l, true);
    if (!validate_solve_layout(P, b->L, b->smw_r, why) || !validate_solve_layout(P, b->L, b->smw_l, why)) {
      free_batch(b);
      return fail(CL_EINVAL, "low-rank solve table check failed: " + why);
    }
    TRY(dalloc(&b->smw_blob_r, b->smw_r.blob.size()));
    HTRY(hipMemcpy(b->smw_blob_r, b->smw_r.blob.data(), b->smw_r.blob.size(), hipMemcpyHostToDevice));
    TRY(dalloc(&b->smw_blob_l, b->smw_l.blob.size()));
    HTRY(hipMemcpy(b->smw_blob_l, b->smw_l.blob.data(), b->smw_l.blob.size(), hipMemcpyHostToDevice));
    // the right and left solves take turns in one workspace
    TRY(dalloc(&b->smw_rhs, (size_t)(std::max(b->smw_r.stride, b->smw_l.stride) * B)));
    TRY(upload(&b->d_pivglob, b->L.pivot_global));
  }
  HTRY(hipMemset(b->status, 0, sizeof(int32_t) * B));
#undef TRY
#undef HTRY
  *out = b;
  return 0;
}

int cl_batch_set_active(cl_batch b, int32_t n) {
  if (!b || n < 1 || n > b->cap) return fail(CL_EINVAL, "active count out of range");
  if (n != b->active) { b->active = n; b->state = 0; }
  return 0;
}

int cl_batch_set_lanes(cl_batch b, int32_t lanes) {
  if (!b || lanes < 0 || lanes > 2) return fail(CL_EINVAL, "lanes must be 0 (automatic), 1 or 2");
  b->lanes = lanes;
  return 0;
}

int cl_batch_use_graph(cl_batch b, int32_t enable) {
  if (!b) return fail(CL_EINVAL, "null batch");
  b->use_graph = enable != 0;
  return 0;
}

int cl_factor(cl_batch b, const void* links_dev, const double* m_host, const double* mu_host) {
  if (!b || !links_dev || !m_host || !mu_host) return fail(CL_EINVAL, "null argument");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = stage_params(b, m_host, mu_host))) return rc;
  if ((rc = enqueue_factor(b, links_dev, false))) return rc;
  b->state = 1;
  return end(b);
}

int cl_selinv(cl_batch b) {
  if (!b) return fail(CL_EINVAL, "null batch");
  if (b->state < 1) return fail(CL_EORDER, "cl_selinv before cl_factor");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_selinv(b))) return rc;
  b->state = 2;
  return end(b);
}

int cl_selected(cl_batch b, void* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 2) return fail(CL_EORDER, "cl_selected before cl_selinv");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_selected(b, out))) return rc;
  return end(b);
}

int cl_drift(cl_batch b, void* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 2) return fail(CL_EORDER, "cl_drift before cl_selinv");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_drift(b, out))) return rc;
  return end(b);
}

int cl_observables(cl_batch b, void* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 2) return fail(CL_EORDER, "cl_observables before cl_selinv");
  int rc;
  if ((rc = begin(b))) return rc;
  const clsel::Plan& P = b->plan->P;
  hipLaunchKernelGGL(clsel::k_observables, dim3(b->active), dim3(256), 0, b->st, b->sel, b->links,
                     b->linv, b->params + b->cap, ldims(P), P.V, (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

int cl_gauge_drift(cl_batch b, const double* beta, void* out) {
  if (!b || !beta || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 1) return fail(CL_EORDER, "cl_gauge_drift before cl_factor");
  for (int i = 0; i < b->active; ++i)
    if (!std::isfinite(beta[i])) return fail(CL_EINVAL, "non-finite beta");
  int rc;
  if ((rc = begin(b))) return rc;
  HIPCHK(hipEventSynchronize(b->ev_lparam));
  for (int i = 0; i < b->active; ++i) b->lparams_host[i] = beta[i];
  HIPCHK(hipMemcpyAsync(b->lparams, b->lparams_host, sizeof(double) * 3 * b->cap,
                        hipMemcpyHostToDevice, b->st));
  HIPCHK(hipEventRecord(b->ev_lparam, b->st));
  const clsel::Plan& P = b->plan->P;
  const dim3 grid((unsigned)cdiv64(P.V * 4, 256), (unsigned)b->active);
  hipLaunchKernelGGL(clsel::k_gauge_drift, grid, dim3(256), 0, b->st, b->links, b->linv,
                     b->lparams, ldims(P), P.V, (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

int cl_langevin_update(cl_batch b, void* links_out, const void* kf, const void* kg,
                       const void* eta, const double* eps_bar, const double* kref, void* eps_out) {
  if (!b || !links_out || !kf || !eta || !eps_bar) return fail(CL_EINVAL, "null argument");
  if (b->state < 1) return fail(CL_EORDER, "cl_langevin_update before cl_factor");
  bool adaptive = false;
  for (int i = 0; i < b->active; ++i) {
    if (!(eps_bar[i] >= 0.0) || !std::isfinite(eps_bar[i])) return fail(CL_EINVAL, "eps_bar must be finite and >= 0");
    if (kref && !std::isfinite(kref[i])) return fail(CL_EINVAL, "non-finite kref");
    adaptive = adaptive || (kref && kref[i] > 0.0);
  }
  int rc;
  if ((rc = begin(b))) return rc;
  HIPCHK(hipEventSynchronize(b->ev_lparam));
  for (int i = 0; i < b->active; ++i) {
    b->lparams_host[b->cap + i] = eps_bar[i];
    b->lparams_host[2 * b->cap + i] = kref ? kref[i] : 0.0;
  }
  HIPCHK(hipMemcpyAsync(b->lparams, b->lparams_host, sizeof(double) * 3 * b->cap,
                        hipMemcpyHostToDevice, b->st));
  HIPCHK(hipEventRecord(b->ev_lparam, b->st));
  const clsel::Plan& P = b->plan->P;
  const dim3 grid((unsigned)cdiv64(P.V * 4, 256), (unsigned)b->active);
  if (adaptive) {
    hipLaunchKernelGGL(k_fill_i32, dim3((2 * b->active + 255) / 256), dim3(256), 0, b->st,
                       (int32_t*)b->kmax, 2 * b->active, 0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(clsel::k_drift_max, grid, dim3(256), 0, b->st, (const double2*)kf,
                       (const double2*)kg, P.V, b->kmax);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(clsel::k_langevin_update, grid, dim3(256), 0, b->st, b->links,
                     (double2*)links_out, (const double2*)kf, (const double2*)kg, (const double*)eta,
                     b->lparams + b->cap, b->lparams + 2 * b->cap, b->kmax, P.V, (double*)eps_out);
  HIPCHK(hipGetLastError());
  return end(b);
}

namespace {
constexpr int kMaxRhs = 4096;

int prepare_solve(cl_batch b, int ns) {
  if (b->solve.ns == ns && b->rhs) return 0;
  const clsel::Plan& P = b->plan->P;
  SolveLayout S;
  build_solve_layout(P, b->L, ns, false, b->L.R, S);
  std::string why;
  if (!validate_solve_layout(P, b->L, S, why)) return fail(CL_EINVAL, "solve table check failed: " + why);
  HIPCHK(hipStreamSynchronize(b->st));  // the old workspace may still be in use
  hipFree(b->solve_blob); b->solve_blob = nullptr;
  hipFree(b->rhs); b->rhs = nullptr;
  b->solve = SolveLayout{};
  int rc;
  if ((rc = dalloc(&b->solve_blob, S.blob.size()))) return rc;
  HIPCHK(hipMemcpy(b->solve_blob, S.blob.data(), S.blob.size(), hipMemcpyHostToDevice));
  if ((rc = dalloc(&b->rhs, (size_t)(S.stride * b->cap)))) return rc;
  b->solve = std::move(S);
  return 0;
}

// Runs the launch tables of one solve: right-hand sides read from in (per-configuration
// stride in_stride, layout [N][ns]), solution written (or added, accumulate) to out.
int run_solve(cl_batch b, const SolveLayout& S, const char* dblob, double2* ws_rhs, const void* in,
              int64_t in_stride, void* out, int64_t out_stride, int accumulate) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active, ns = S.ns;
  const int64_t stride = S.stride;
  const int32_t* lim = S.live ? b->iws + b->L.cnt_off : nullptr;
  const int64_t lst = b->L.iws_elems;
  auto run = [&](const Launch& l) -> int {
    if (l.gridx <= 0) return 0;
    const dim3 grid((unsigned)l.gridx, (unsigned)B);
    const char* dp = dblob + l.desc_off;
    switch (l.kind) {
      case kRhsAsm:
        if (l.rpt)
          hipLaunchKernelGGL(clsel::k_rhs_assemble<true>, grid, dim3(256), 0, b->st, (const clsel::RhsAsmDesc*)dp,
                             l.count, ws_rhs, stride, (const double2*)in, in_stride, b->d_front_sites, b->d_inv, ns,
                             lim, lst);
        else
          hipLaunchKernelGGL(clsel::k_rhs_assemble<false>, grid, dim3(256), 0, b->st, (const clsel::RhsAsmDesc*)dp,
                             l.count, ws_rhs, stride, (const double2*)in, in_stride, b->d_front_sites, b->d_inv, ns,
                             lim, lst);
        break;
      case kRhsGather:
        if (l.rpt)
          hipLaunchKernelGGL(clsel::k_rhs_gather<true>, grid, dim3(256), 0, b->st, (const clsel::RhsGatherDesc*)dp,
                             l.count, ws_rhs, stride, b->d_rel, ns, lim, lst);
        else
          hipLaunchKernelGGL(clsel::k_rhs_gather<false>, grid, dim3(256), 0, b->st, (const clsel::RhsGatherDesc*)dp,
                             l.count, ws_rhs, stride, b->d_rel, ns, lim, lst);
        break;
      case kSolScatter:
        if (l.rpt)
          hipLaunchKernelGGL(clsel::k_sol_scatter<true>, grid, dim3(256), 0, b->st, (const clsel::SolScatterDesc*)dp,
                             l.count, ws_rhs, stride, (double2*)out, out_stride, b->d_front_sites, ns, accumulate,
                             lim, lst);
        else
          hipLaunchKernelGGL(clsel::k_sol_scatter<false>, grid, dim3(256), 0, b->st, (const clsel::SolScatterDesc*)dp,
                             l.count, ws_rhs, stride, (double2*)out, out_stride, b->d_front_sites, ns, accumulate,
                             lim, lst);
        break;
      default:
        clsel::launch_gemm(l.rpt, l.tile, grid, b->st, (const clsel::GemmDesc*)dp, l.count, b->fronts,
                           b->L.cfg_stride, P.pool_elems, b->ws, b->L.ws_elems, b->iws, b->L.iws_elems,
                           ws_rhs, stride, b->d_inv, (double2*)out, out_stride, true, lim, lst);
    }
    HIPCHK(hipGetLastError());
    return 0;
  };
  int rc;
  for (const Launch& l : S.fwd) if ((rc = run(l))) return rc;
  for (const Launch& l : S.bwd) if ((rc = run(l))) return rc;
  return run(S.scatter);
}

clsel::SmwCtx smw_ctx(cl_batch b) {
  const Layout& L = b->L;
  clsel::SmwCtx c{};
  c.ws = b->ws; c.ws_stride = L.ws_elems;
  c.iws = b->iws; c.iws_stride = L.iws_elems;
  c.pdelta_off = L.pdelta_off; c.x_off = L.x_off; c.y_off = L.y_off; c.xc_off = L.xc_off;
  c.r_off = L.r_off; c.c_off = L.c_off; c.dl_off = L.dl_off;
  c.peq_off = L.peq_off; c.li_off = L.li_off; c.lj_off = L.lj_off; c.cnt_off = L.cnt_off;
  c.pivot_global = b->d_pivglob;
  c.n = b->plan->P.N;
  c.R = L.R;
  c.status = b->status;
  return c;
}

// The low-rank correction of the perturbed pivots, after the selected blocks of D~ are
// gathered (see k_smw.hip): X and Y^T by right and left solves (with the plan's
// smw_refine, one refinement step each), C = (I + V^T X)^{-1}, X C, and the blocks
// corrected in place.
int enqueue_smw(cl_batch b) {
  const clsel::Plan& P = b->plan->P;
  const Layout& L = b->L;
  if (L.R == 0) return 0;
  const int B = b->active;
  const clsel::SmwCtx c = smw_ctx(b);
  const dim3 g_nr((unsigned)cdiv64(P.N * L.R, 256), (unsigned)B);
  const dim3 g_vr((unsigned)cdiv64(P.V * L.R, 256), (unsigned)B);
  const dim3 g_rr((unsigned)cdiv64((int64_t)L.R * L.R, 256), (unsigned)B);
  double2* rbuf = b->ws + L.r_off;
  double2* X = b->ws + L.x_off;
  double2* Yt = b->ws + L.y_off;
  const int64_t wst = L.ws_elems;
  int rc;
  // X = D~^{-1} U, Y^T = D~^{-T} V
  hipLaunchKernelGGL(clsel::k_smw_rhs, g_nr, dim3(256), 0, b->st, c, 0);
  HIPCHK(hipGetLastError());
  if ((rc = run_solve(b, b->smw_r, b->smw_blob_r, b->smw_rhs, rbuf, wst, X, wst, 0))) return rc;
  hipLaunchKernelGGL(clsel::k_smw_rhs, g_nr, dim3(256), 0, b->st, c, 1);
  HIPCHK(hipGetLastError());
  if ((rc = run_solve(b, b->smw_l, b->smw_blob_l, b->smw_rhs, rbuf, wst, Yt, wst, 0))) return rc;
  // optionally one refinement step each: residual against D~ = D + perturbations, solve, add
  for (int trans = 0; trans < 2 * P.opt.smw_refine; ++trans) {
    hipLaunchKernelGGL(clsel::k_smw_residual, g_vr, dim3(256), 0, b->st, c, b->links, b->linv, b->params,
                       b->params + b->cap, ldims(P), P.V, trans);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(clsel::k_smw_residual_delta, g_rr, dim3(256), 0, b->st, c, trans);
    HIPCHK(hipGetLastError());
    if ((rc = run_solve(b, trans ? b->smw_l : b->smw_r, trans ? b->smw_blob_l : b->smw_blob_r, b->smw_rhs,
                        rbuf, wst, trans ? Yt : X, wst, 1)))
      return rc;
  }
  hipLaunchKernelGGL(clsel::k_smw_capacitance, dim3(B), dim3(1024), 0, b->st, c);
  HIPCHK(hipGetLastError());
  clsel::launch_gemm(0, L.smw_xc.tile, dim3((unsigned)L.smw_xc.gridx, (unsigned)B), b->st,
                     (const clsel::GemmDesc*)(b->dblob + L.smw_xc.desc_off), L.smw_xc.count, b->fronts,
                     L.cfg_stride, P.pool_elems, b->ws, L.ws_elems, b->iws, L.iws_elems, nullptr, 0, b->d_inv,
                     nullptr, 0, true, b->iws + L.cnt_off, L.iws_elems);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(clsel::k_smw_correct, dim3((unsigned)cdiv64(P.V * 9, 256), (unsigned)B), dim3(256), 0,
                     b->st, c, b->sel, ldims(P), P.V);
  HIPCHK(hipGetLastError());
  return 0;
}

int enqueue_solve(cl_batch b, const void* rhs_dev, void* x_dev) {
  const clsel::Plan& P = b->plan->P;
  const SolveLayout& S = b->solve;
  const int64_t vstride = P.N * (int64_t)S.ns;
  int rc;
  if ((rc = run_solve(b, S, b->solve_blob, b->rhs, rhs_dev, vstride, x_dev, vstride, 0))) return rc;
  if (b->L.R == 0) return 0;
  // x -= X C (V^T x): the solution of D~ corrected to that of D
  const clsel::SmwCtx c = smw_ctx(b);
  const int B = b->active;
  hipLaunchKernelGGL(clsel::k_smw_gather_rows, dim3((unsigned)cdiv64((int64_t)b->L.R * S.ns, 256), (unsigned)B),
                     dim3(256), 0, b->st, c, (const double2*)x_dev, vstride, b->rhs + S.t_off, S.stride, S.ns);
  HIPCHK(hipGetLastError());
  clsel::launch_gemm(0, S.corr.tile, dim3((unsigned)S.corr.gridx, (unsigned)B), b->st,
                     (const clsel::GemmDesc*)(b->solve_blob + S.corr.desc_off), S.corr.count, b->fronts,
                     b->L.cfg_stride, P.pool_elems, b->ws, b->L.ws_elems, b->iws, b->L.iws_elems, b->rhs,
                     S.stride, b->d_inv, (double2*)x_dev, vstride, true);
  HIPCHK(hipGetLastError());
  return 0;
}
}  // namespace

int cl_solve(cl_batch b, const void* rhs_dev, int32_t ns, void* x_dev) {
  if (!b || !rhs_dev || !x_dev) return fail(CL_EINVAL, "null argument");
  if (ns < 1 || ns > kMaxRhs) return fail(CL_EINVAL, "right-hand sides must be 1 .. 4096");
  if (b->state < 1) return fail(CL_EORDER, "cl_solve before cl_factor");
  if (b->L.R > 0 && b->state < 2)
    return fail(CL_EORDER, "cl_solve before cl_selinv (the perturbed pivots' correction comes from it)");
  int rc;
  HIPCHK(hipSetDevice(b->device));
  if ((rc = prepare_solve(b, ns))) return rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_solve(b, rhs_dev, x_dev))) return rc;
  return end(b);
}

int cl_stochastic_blocks(cl_batch b, const void* xi_dev, const void* x_dev, int32_t ns, void* out) {
  if (!b || !xi_dev || !x_dev || !out) return fail(CL_EINVAL, "null argument");
  if (ns < 1 || ns > kMaxRhs) return fail(CL_EINVAL, "samples must be 1 .. 4096");
  if (b->state < 1) return fail(CL_EORDER, "cl_stochastic_blocks before cl_factor");
  int rc;
  if ((rc = begin(b))) return rc;
  const clsel::Plan& P = b->plan->P;
  const dim3 grid((unsigned)cdiv64(P.V * 81, 256), (unsigned)b->active);
  hipLaunchKernelGGL(clsel::k_stochastic_blocks, grid, dim3(256), 0, b->st, (const double2*)x_dev,
                     (const double2*)xi_dev, ldims(P), P.V, ns, (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

int cl_drift_from_blocks(cl_batch b, const void* blocks_dev, void* out) {
  if (!b || !blocks_dev || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 1) return fail(CL_EORDER, "cl_drift_from_blocks before cl_factor");
  int rc;
  if ((rc = begin(b))) return rc;
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  const int64_t n = P.V * 4 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_drift, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, b->st,
                     (const double2*)blocks_dev, b->links, b->linv, b->params + b->cap, ldims(P), P.V, B,
                     (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

}  // extern "C"

// ------------------------------------------------------------ no-allocation entry point
// The workspaces of cl_run_noalloc live in this array. Host code never passes its name to
// a kernel or a copy (on the host the name is only a stand-in): it takes the device
// address with hipGetSymbolAddress, once per device with that device current, and uses
// that address everywhere.
static __device__ __align__(256) unsigned char scratch[CL_NOALLOC_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

int scratch_address(int device, char** out) {
  if (device < 0 || device >= 64) return fail(CL_ENODEV, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = (char*)g_scratch_ptr[device];
  return 0;
}

// Carves 256-byte aligned pieces out of the scratch array.
struct Carver {
  char* base;
  size_t used = 0;
  template <class T>
  T* take(size_t n) {
    used = (used + 255) & ~size_t(255);
    T* p = (T*)(base + used);
    used += (n ? n : 1) * sizeof(T);
    return p;
  }
};

}  // namespace

extern "C" {

int cl_run_noalloc(cl_plan plan, int32_t batch, const void* links_dev, const double* m_host,
                   const double* mu_host, void* sel_out, void* drift_out, int32_t* status_host,
                   void* hip_stream) {
  if (!plan || !links_dev || !m_host || !mu_host || !status_host || batch < 1 || batch > 65535)
    return fail(CL_EINVAL, "null argument or batch out of range");
  const clsel::Plan& P = plan->P;
  int device = 0;
  HIPCHK(hipGetDevice(&device));
  // the same tables and launch lists a batch builds, on the host
  cl_batch_s b;
  b.plan = plan;
  b.cap = b.active = batch;
  b.device = device;
  b.st = b.user = (hipStream_t)hip_stream;
  build_layout(P, b.L);
  std::string why;
  if (!validate_layout(P, b.L, why)) return fail(CL_EINVAL, "launch table check failed: " + why);
  if (b.L.R > 0) {
    build_solve_layout(P, b.L, b.L.R, false, 0, b.smw_r, true);
    build_solve_layout(P, b.L, b.L.R, true, 0, b.smw_l, true);
    if (!validate_solve_layout(P, b.L, b.smw_r, why) || !validate_solve_layout(P, b.L, b.smw_l, why))
      return fail(CL_EINVAL, "low-rank solve table check failed: " + why);
  }
  char* base = nullptr;
  int rc;
  if ((rc = scratch_address(device, &base))) return rc;
  const int64_t B = batch;
  Carver c{base};
  b.dblob = c.take<char>(b.L.blob.size());
  b.d_front_sites = c.take<int32_t>(P.front_sites.size());
  b.d_site_coords = c.take<int32_t>(P.site_coords.size());
  b.d_inv = c.take<int32_t>(P.inv_maps.size());
  b.d_rel = c.take<int32_t>(P.rel_maps.size());
  b.d_sel_off = c.take<int64_t>(P.sel_off.size());
  b.d_sel_ld = c.take<int32_t>(P.sel_ld.size());
  b.params = c.take<double>(2 * B);
  b.status = c.take<int32_t>(B);
  b.fronts = c.take<double2>(B * b.L.cfg_stride);
  b.ws = c.take<double2>(B * b.L.ws_elems);
  b.iws = c.take<int32_t>(B * b.L.iws_elems);
  b.links = c.take<double2>(B * b.L.links_elems);
  b.linv = c.take<double2>(B * b.L.links_elems);
  b.sel = c.take<double2>(B * b.L.sel_elems);
  if (b.L.R > 0) {
    b.smw_blob_r = c.take<char>(b.smw_r.blob.size());
    b.smw_blob_l = c.take<char>(b.smw_l.blob.size());
    b.smw_rhs = c.take<double2>(B * b.smw_r.stride);
    b.d_pivglob = c.take<int32_t>(b.L.pivot_global.size());
  }
  if (c.used > (size_t)CL_NOALLOC_BYTES)
    return fail(CL_EINVAL, "cl_run_noalloc: this plan and batch need " + std::to_string(c.used) +
                               " bytes of workspace; the static array holds " +
                               std::to_string((size_t)CL_NOALLOC_BYTES));
  // tables and parameters into the array (from host memory that lives until the final wait)
  std::vector<double> params(2 * B);
  for (int64_t i = 0; i < B; ++i) { params[i] = m_host[i]; params[B + i] = mu_host[i]; }
  auto put = [&](void* dst, const void* src, size_t n) -> int {
    if (n) HIPCHK(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, b.st));
    return 0;
  };
  if ((rc = put(b.dblob, b.L.blob.data(), b.L.blob.size())) ||
      (rc = put(b.d_front_sites, P.front_sites.data(), P.front_sites.size() * 4)) ||
      (rc = put(b.d_site_coords, P.site_coords.data(), P.site_coords.size() * 4)) ||
      (rc = put(b.d_inv, P.inv_maps.data(), P.inv_maps.size() * 4)) ||
      (rc = put(b.d_rel, P.rel_maps.data(), P.rel_maps.size() * 4)) ||
      (rc = put(b.d_sel_off, P.sel_off.data(), P.sel_off.size() * 8)) ||
      (rc = put(b.d_sel_ld, P.sel_ld.data(), P.sel_ld.size() * 4)))
    return rc;
  if (b.L.R > 0 &&
      ((rc = put(b.smw_blob_r, b.smw_r.blob.data(), b.smw_r.blob.size())) ||
       (rc = put(b.smw_blob_l, b.smw_l.blob.data(), b.smw_l.blob.size())) ||
       (rc = put(b.d_pivglob, b.L.pivot_global.data(), b.L.pivot_global.size() * 4))))
    return rc;
  // the parameters go straight to the array (a batch stages them in pinned memory)
  b.params_host = params.data();
  if ((rc = enqueue_factor(&b, links_dev, true)) || (rc = enqueue_selinv(&b)) ||
      (sel_out && (rc = enqueue_selected(&b, sel_out))) || (drift_out && (rc = enqueue_drift(&b, drift_out))))
    return rc;
  HIPCHK(hipMemcpyAsync(status_host, b.status, sizeof(int32_t) * B, hipMemcpyDeviceToHost, b.st));
  HIPCHK(hipStreamSynchronize(b.st));
  b.params_host = nullptr;
  return 0;
}

int cl_run(cl_batch b, const void* links_dev, const double* m_host, const double* mu_host,
           void* sel_out, void* drift_out) {
  if (!b || !links_dev || !m_host || !mu_host) return fail(CL_EINVAL, "null argument");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = stage_params(b, m_host, mu_host))) return rc;
  if (!b->use_graph) {
    if ((rc = enqueue_run(b, links_dev, sel_out, drift_out, false))) return rc;
  } else {
    if (!b->gexec || b->g_links != links_dev || b->g_sel != sel_out || b->g_drift != drift_out ||
        b->g_active != b->active || b->g_lanes != run_lanes(b)) {
      if (b->gexec) { hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
      HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
      rc = enqueue_run(b, links_dev, sel_out, drift_out, true);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(b->st, &graph);
      if (rc) { if (graph) hipGraphDestroy(graph); return rc; }
      if (e != hipSuccess) return fail(CL_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (e != hipSuccess) { b->gexec = nullptr; return fail(CL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)); }
      b->g_links = links_dev; b->g_sel = sel_out; b->g_drift = drift_out; b->g_active = b->active;
      b->g_lanes = run_lanes(b);
    }
    HIPCHK(hipGraphLaunch(b->gexec, b->st));
    HIPCHK(hipEventRecord(b->ev_param, b->st));
  }
  b->state = 2;
  return end(b);
}

int cl_batch_profile(cl_batch b, int32_t gemm_modes) {
  if (!b) return fail(CL_EINVAL, "null batch");
  if (gemm_modes < 0 || gemm_modes > 7) return fail(CL_EINVAL, "gemm_modes is a mask of bits 0..2");
  if (gemm_modes && b->use_graph) return fail(CL_EINVAL, "profiling needs the eager path");
  b->prof = gemm_modes;
  return 0;
}

int cl_batch_profile_read(cl_batch b, double* gemm_ms, double* gemm_flops, double* gemm_bytes,
                          int64_t* launches) {
  if (!b || !gemm_ms || !gemm_flops || !gemm_bytes || !launches)
    return fail(CL_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(b->st));
  for (size_t i = 0; i + 1 < b->prof_used; i += 2) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, b->prof_ev[i], b->prof_ev[i + 1]));
    b->prof_ms += ms;
    b->prof_flop_total += b->prof_flops[i / 2];
    b->prof_byte_total += b->prof_bytes[i / 2];
    ++b->prof_launches;
  }
  b->prof_used = 0;
  b->prof_flops.clear();
  b->prof_bytes.clear();
  b->prof_mode.clear();
  *gemm_ms = b->prof_ms;
  *gemm_flops = b->prof_flop_total;
  *gemm_bytes = b->prof_byte_total;
  *launches = b->prof_launches;
  b->prof_ms = 0;
  b->prof_flop_total = 0;
  b->prof_byte_total = 0;
  b->prof_launches = 0;
  return 0;
}

int cl_batch_profile_launches(cl_batch b, int64_t cap, double* ms, double* flops, double* bytes,
                              int32_t* mode, int64_t* n) {
  if (!b || !n || cap < 0 || (cap > 0 && (!ms || !flops || !bytes || !mode)))
    return fail(CL_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(b->st));
  const int64_t timed = (int64_t)(b->prof_used / 2);
  for (int64_t i = 0; i < timed && i < cap; ++i) {
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, b->prof_ev[2 * i], b->prof_ev[2 * i + 1]));
    ms[i] = t;
    flops[i] = b->prof_flops[i];
    bytes[i] = b->prof_bytes[i];
    mode[i] = b->prof_mode[i];
  }
  *n = timed;
  return 0;
}

int cl_status(cl_batch b, int32_t* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipStreamSynchronize(b->st));
  HIPCHK(hipMemcpy(out, b->status, sizeof(int32_t) * b->active, hipMemcpyDeviceToHost));
  return 0;
}

int cl_batch_inject_fault(cl_batch b, int32_t config, int32_t front) {
  if (!b) return fail(CL_EINVAL, "null batch");
  if (front >= (int32_t)b->plan->P.fronts.size() || config >= b->cap)
    return fail(CL_EINVAL, "front or configuration out of range");
  b->fault_cfg = front < 0 ? -1 : config;
  b->fault_front = front < 0 ? -1 : front;
  if (b->gexec) { hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }  // recapture with it
  return 0;
}

int cl_batch_perturbations(cl_batch b, int32_t* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipStreamSynchronize(b->st));
  for (int i = 0; i < b->active; ++i) {
    out[i] = 0;
    if (b->L.R > 0)
      HIPCHK(hipMemcpy(out + i, b->iws + (int64_t)i * b->L.iws_elems + b->L.cnt_off + 1, sizeof(int32_t),
                       hipMemcpyDeviceToHost));
  }
  return 0;
}

int cl_batch_query(cl_batch b) {
  if (!b) return fail(CL_EINVAL, "null batch");
  HIPCHK(hipSetDevice(b->device));
  const hipError_t e = hipEventQuery(b->ev_out);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return fail(CL_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
}

int cl_batch_sync(cl_batch b) {
  if (!b) return fail(CL_EINVAL, "null batch");
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipStreamSynchronize(b->st));
  return 0;
}

void cl_batch_destroy(cl_batch b) {
  if (!b) return;
  hipSetDevice(b->device);
  hipStreamSynchronize(b->st);
  free_batch(b);
}

}  // extern "C"
