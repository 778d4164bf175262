// C ABI of libhfd (declared in include/hfd.h): context life cycle, device
// memory, the geometric precompute and the hot-path launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hfd.h"
#include "kernels.h"
#include "setup.h"

// Stage a two-lane edge-pass block's stencil rows in LDS (0: gather every
// node from HBM).
#ifndef HFD_EDGE_STAGE
#define HFD_EDGE_STAGE 1
#endif
// Stage a vertex-pass block's neighbour data in LDS (0: gather every slot
// from HBM).
#ifndef HFD_VERTEX_STAGE
#define HFD_VERTEX_STAGE 1
#endif

using hfd::GasParams;

// Degree of the inviscid divergence fit when the caller does not choose one.
#ifndef HFD_DEFAULT_DEG_INV
#define HFD_DEFAULT_DEG_INV 5
#endif

// Scratch of hfd_stable_dt_noalloc: the per-block partial minima of the time
// step (one per 256 owned vertices).  A file-scope device array: every GPU
// the library runs on holds its own copy until the process ends.  Host code
// never passes this name to a kernel; it uses the per-device address that
// hipGetSymbolAddress returns (scratch_setup below).
constexpr int64_t kNoallocDtPartials = 16384;
static __device__ __align__(256) double scratch[kNoallocDtPartials];

struct hfd_ctx {
  hfd_opts o{};
  int device = -1;
  std::string err;
  hfd::HostSetup hs;
  hfd_info info{};
  std::vector<void*> allocs;

  // float64 coefficients
  int32_t* stg = nullptr;
  // staging lists of the two-lane edge kernel (null: not staged)
  int32_t *erp = nullptr, *erow = nullptr;
  uint16_t* epos = nullptr;
  int e_max_rows = 0;
  double *n = nullptr, *w5 = nullptr, *w3 = nullptr;
  double *w5g = nullptr, *w3g = nullptr;  // midpoint-derivative rows (edge_grad)
  uint8_t* gmask = nullptr;               // branch mask for them when none is asked
  int32_t* rank = nullptr;
  int8_t* trunc3 = nullptr;
  int32_t *vptr = nullptr, *eptr = nullptr, *vg = nullptr, *ve = nullptr;
  double *dv = nullptr, *de = nullptr, *dvis = nullptr;
  // LDS staging lists of the vertex pass (host copies live until upload)
  struct Stage {
    std::vector<int32_t> rp, rows, ep, edges;
    std::vector<uint16_t> vloc, eloc;
    std::vector<uint32_t> base;
    int max_rows = 0, max_edges = 0, idx_bytes = 0;
    int64_t list_ints = 0;  // 4-byte entries of rp, rows, ep, edges and base
  } stage;
  int32_t *hrp = nullptr, *hrow = nullptr, *hep = nullptr, *hedge = nullptr;
  uint32_t* lbase = nullptr;
  void *vloc = nullptr, *eloc = nullptr;
  double* hmin = nullptr;
  int32_t *dir_rows = nullptr, *copy_rows = nullptr, *copy_src = nullptr;
  // float32 copies (mixed form)
  float *fn = nullptr, *fw5 = nullptr, *fw3 = nullptr, *fdv = nullptr,
        *fde = nullptr, *fdvis = nullptr;
  // work buffers: float64 Runge-Kutta stage states [12][nv], and per
  // precision the gather-layout stage states and the edge fluxes
  double *U1 = nullptr, *U2 = nullptr;
  template <class T>
  struct Bufs {
    hfd::V4<T>* Gv[3] = {nullptr, nullptr, nullptr};
    hfd::V4<T>* Gg[3] = {nullptr, nullptr, nullptr};
    hfd::V4<T>* H = nullptr;
  };
  Bufs<double> b64;
  Bufs<float> b32;
  double* dtpart = nullptr;
  int64_t ndtpart = 0;
  double* scratch_dev = nullptr;  // this device's address of `scratch`
  int32_t* flag = nullptr;
  const uint8_t* force = nullptr;
  // adjoint: transposed maps and work buffers (built at first use)
  bool adj_ready = false;
  bool adj_coef_ready = false;  // de_t, dv_t, dvis_t match the current coefficients
  int32_t *etp = nullptr, *etv = nullptr, *ets = nullptr;
  int32_t *alrp = nullptr, *alrow = nullptr;  // staging lists of the edge reverse
  uint16_t* alpos = nullptr;
  int32_t *vtp = nullptr, *vtv = nullptr, *vts = nullptr;
  int32_t *ntp = nullptr, *nte = nullptr;
  int8_t* ntj = nullptr;
  int32_t *gsp = nullptr, *gsr = nullptr, *gsg = nullptr;  // copy source -> ghosts
  int64_t n_gsrc = 0;
  double *bnode = nullptr, *AL1 = nullptr, *AL2 = nullptr, *AL3 = nullptr;
  uint8_t* adj_mask = nullptr;  // the forward's switch decisions at the state being reversed
  double *de_t = nullptr, *dv_t = nullptr, *dvis_t = nullptr;  // rows in transposed order
  // float32 adjoint (mixed form, allocated at its first use)
  bool adj_coef32_ready = false;             // fde_t, fdv_t match de_t, dv_t
  float *fde_t = nullptr, *fdv_t = nullptr, *fdvis_t = nullptr, *bnode32 = nullptr;
  hfd::V4<float>* LGv32[2] = {nullptr, nullptr};  // lambda in gather layout,
  hfd::V4<float>* LGg32[2] = {nullptr, nullptr};  // two for successive stages
  hfd::V4<double>* LGv[2] = {nullptr, nullptr};
  hfd::V4<double>* LGg[2] = {nullptr, nullptr};
  // measurement: event pairs around the edge (0) and vertex (1) passes
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[2];
};

namespace {

thread_local std::string g_create_err;  // message of the last failed hfd_create

hfd_status fail(hfd_ctx* c, hfd_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(ctx, expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, HFD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
hfd_status dalloc(hfd_ctx* c, T** p, int64_t n) {
  *p = nullptr;
  if (n <= 0) return HFD_OK;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, size_t(n) * sizeof(T));
  if (e != hipSuccess)
    return fail(c, HFD_E_NOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) +
                                    " bytes: " + hipGetErrorString(e));
  c->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return HFD_OK;
}

template <class T, class A>
hfd_status upload(hfd_ctx* c, T** p, const std::vector<T, A>& h) {
  hfd_status s = dalloc(c, p, int64_t(h.size()));
  if (s != HFD_OK) return s;
  if (!h.empty()) HIPCHK(c, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return HFD_OK;
}

void dfree(hfd_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  hipFree(p);
}

GasParams gas_params(const hfd_ctx* c, bool mixed) {
  GasParams g{};
  g.gamma = c->o.gamma;
  g.gas_R = c->o.gas_R;
  g.mu = c->o.mu;
  g.prandtl = c->o.prandtl;
  g.eps = c->o.weno_eps;
  g.sw_lo = c->o.sw_lo;
  g.sw_hi = c->o.sw_hi;
  for (int q = 0; q < 4; ++q) g.wref[q] = mixed ? c->o.w_ref[q] : 0.0;
  const double rho = g.wref[0];
  g.uref = rho > 0 ? g.wref[1] / rho : 0.0;
  g.vref = rho > 0 ? g.wref[2] / rho : 0.0;
  const double p = (g.gamma - 1.0) * (g.wref[3] - 0.5 * rho * (g.uref * g.uref + g.vref * g.vref));
  g.etr_ref = g.wref[3] + p;
  g.sw = c->o.switch_mode;
  g.flux = c->o.flux;
  g.f_gamma = float(g.gamma);
  g.f_gm1 = float(g.gamma - 1.0);
  g.f_eps = float(g.eps);
  g.f_sw_lo = float(g.sw_lo);
  g.f_sw_hi = float(g.sw_hi);
  for (int q = 0; q < 4; ++q) g.f_wref[q] = float(g.wref[q]);
  g.f_uref = float(g.uref);
  g.f_vref = float(g.vref);
  g.f_etr_ref = float(g.etr_ref);
  return g;
}

bool mixed(const hfd_ctx* c) { return c->o.precision == HFD_FP32_MIXED; }

// One staging list family: for each block of kStageVertices owned vertices
// (slots ptr[v0] .. ptr[v0 + 16]), the sorted distinct ids its slots name
// (list[bp[b] .. bp[b+1])); per vertex the first list position among its
// slots (base), per slot its position minus its vertex's base (loc).
// longest: longest list; span: largest loc + 1.
template <class A>
void stage_lists(const std::vector<int64_t>& ptr, const std::vector<int32_t, A>& ids,
                 int64_t nowned, std::vector<int32_t>& bp, std::vector<int32_t>& list,
                 std::vector<uint16_t>& base, std::vector<uint16_t>& loc, int& longest,
                 int& span) {
  const int64_t vpb = hfd::kStageVertices, nb = (nowned + vpb - 1) / vpb;
  std::vector<std::vector<int32_t>> blists;
  blists.resize(size_t(nb));
  base.assign(size_t(nowned), 0);
  loc.assign(ids.size(), 0);
  int tl[16] = {0}, ts[16] = {0};
  hfd::parallel_for(nb, [&](int64_t b0, int64_t b1, unsigned t) {
    std::vector<uint64_t> key;
    std::vector<int32_t> pos;
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t v0 = b * vpb, v1 = std::min(nowned, v0 + vpb), k0 = ptr[v0];
      const int64_t n = ptr[v1] - k0;
      // (id, slot) pairs in id order give each slot its list position
      key.resize(size_t(n));
      pos.resize(size_t(n));
      for (int64_t k = 0; k < n; ++k) key[k] = (uint64_t(uint32_t(ids[k0 + k])) << 32) | uint64_t(k);
      std::sort(key.begin(), key.end());
      std::vector<int32_t>& blk = blists[b];
      blk.clear();
      for (int64_t i = 0; i < n; ++i) {
        const int32_t u = int32_t(key[i] >> 32);
        if (blk.empty() || blk.back() != u) blk.push_back(u);
        pos[key[i] & 0xffffffffu] = int32_t(blk.size()) - 1;
      }
      for (int64_t v = v0; v < v1; ++v) {
        int32_t lo = INT32_MAX;
        for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k) lo = std::min(lo, pos[k - k0]);
        if (ptr[v + 1] == ptr[v]) lo = 0;
        base[v] = uint16_t(lo);
        for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k) {
          const int32_t d = pos[k - k0] - lo;
          loc[k] = uint16_t(d);
          ts[t] = std::max(ts[t], d + 1);
        }
      }
      tl[t] = std::max(tl[t], int(blk.size()));
    }
  });
  longest = *std::max_element(tl, tl + 16);
  span = *std::max_element(ts, ts + 16);
  bp.assign(size_t(nb + 1), 0);
  for (int64_t b = 0; b < nb; ++b) bp[b + 1] = bp[b] + int32_t(blists[b].size());
  list.resize(size_t(bp[nb]));
  for (int64_t b = 0; b < nb; ++b) std::copy(blists[b].begin(), blists[b].end(), list.begin() + bp[b]);
}

// Staging lists of the vertex pass, kept when a block's data fits in LDS
// (float64 values, gradients with viscosity, and fluxes).  Local ids take
// one byte when every vertex's slots span at most 256 list positions.
void build_stage(hfd_ctx* c) {
  auto& g = c->stage;
  g = hfd_ctx::Stage{};
  const hfd::HostSetup& h = c->hs;
  if (!HFD_VERTEX_STAGE || c->o.stage_off || h.n_owned == 0) return;
  std::vector<uint16_t> rb, eb;
  int rspan = 0, espan = 0;
  stage_lists(h.vptr, h.v_gather, h.n_owned, g.rp, g.rows, rb, g.vloc, g.max_rows, rspan);
  stage_lists(h.eptr, h.v_edges, h.n_owned, g.ep, g.edges, eb, g.eloc, g.max_edges, espan);
  const int64_t lds = ((c->o.mu > 0.0 ? 3 : 1) * int64_t(g.max_rows) + g.max_edges) * 32;
  if (lds > 48 * 1024 || g.max_rows > 65536 || g.max_edges > 65536) {
    g = hfd_ctx::Stage{};
    return;
  }
  g.base.resize(size_t(h.n_owned));
  for (int64_t v = 0; v < h.n_owned; ++v) g.base[v] = uint32_t(rb[v]) | (uint32_t(eb[v]) << 16);
  g.idx_bytes = (rspan <= 256 && espan <= 256) ? 1 : 2;
  g.list_ints = int64_t(g.rp.size() + g.ep.size() + g.rows.size() + g.edges.size() +
                        g.base.size());
}

// Staging lists of the two-lane edge kernel: per block of kEdgeStageEdges
// consecutive edges the sorted distinct rows of their six stencil nodes,
// and per stencil node (SoA [6][ne]) its position in its block's list.
// Empty when a block's rows would not fit the LDS budget.
void edge_stage_lists(const hfd::HostSetup& h, std::vector<int32_t>& rp,
                      std::vector<int32_t>& rows, std::vector<uint16_t>& pos, int& longest) {
  const int64_t ne = h.ne, eb = hfd::kEdgeStageEdges, nb = (ne + eb - 1) / eb;
  std::vector<std::vector<int32_t>> bl;
  bl.resize(size_t(nb));
  pos.assign(size_t(6 * ne), 0);
  int tl[16] = {0};
  hfd::parallel_for(nb, [&](int64_t b0, int64_t b1, unsigned t) {
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t e0 = b * eb, e1 = std::min(ne, e0 + eb);
      std::vector<int32_t>& L = bl[size_t(b)];
      L.clear();
      for (int j = 0; j < 6; ++j)
        for (int64_t e = e0; e < e1; ++e) L.push_back(h.e_stg[j * ne + e]);
      std::sort(L.begin(), L.end());
      L.erase(std::unique(L.begin(), L.end()), L.end());
      for (int j = 0; j < 6; ++j)
        for (int64_t e = e0; e < e1; ++e)
          pos[size_t(j * ne + e)] = uint16_t(
              std::lower_bound(L.begin(), L.end(), h.e_stg[j * ne + e]) - L.begin());
      tl[t] = std::max(tl[t], int(L.size()));
    }
  });
  longest = *std::max_element(tl, tl + 16);
  // 3 records of 4 float64 per row; 64 KB of LDS at most
  if (longest * 3 * 32 > 64 * 1024) {
    rp.clear();
    rows.clear();
    pos.clear();
    longest = 0;
    return;
  }
  rp.assign(size_t(nb + 1), 0);
  for (int64_t b = 0; b < nb; ++b) rp[b + 1] = rp[b] + int32_t(bl[size_t(b)].size());
  rows.resize(size_t(rp[nb]));
  for (int64_t b = 0; b < nb; ++b)
    std::copy(bl[size_t(b)].begin(), bl[size_t(b)].end(), rows.begin() + rp[b]);
}

void byte_model(hfd_ctx* c) {
  hfd_info& I = c->info;
  const double s = mixed(c) ? 4.0 : 8.0;
  const double ne = double(I.n_edges), nv = double(I.nv), no = double(I.n_owned);
  const double visc = c->o.mu > 0.0 ? 1.0 : 0.0;
  // edge pass: ids, direction + Hermite + 3-node weights, the stage state
  // (12 values per vertex), flux out.  Both kernels read the 3-node rows of
  // a side only when the side takes that branch somewhere: those bytes are
  // per side (data-dependent).  With WENO everywhere they are always read,
  // and neither the Hermite rows nor the gradients are.
  const bool w3_lazy = c->o.switch_mode != HFD_SWITCH_WENO_ONLY;
  const double rows = w3_lazy ? 32 : 20;  // direction (2) + Hermite (30) | 3-node (18)
  const double state = w3_lazy ? 12 : 4;
  I.bytes_edge_launch = ne * (6 * 4 + rows * s + 4 * s) + nv * state * s;
  I.bytes_edge_w3_side = w3_lazy ? 9 * s : 0.0;
  // vertex pass: CSR offsets and ids, coefficient records, state (values,
  // plus gradients with viscosity), edge fluxes, float64 RK update
  // averaged over the three stages: U^n read and U^new written every stage,
  // U^k read in stages 2 and 3, the gather-layout copy of the new state
  // written every stage (by the last one when hfd_rk_steps continues with
  // another step)
  double rk = no * (2 * 96.0 + (2.0 / 3.0) * 96.0 + 12 * s);
  I.bytes_vertex_launch = (no + 1) * 8 + double(I.n_vslots) * (4 + 6 * s + visc * 5 * s) +
                          double(I.n_eslots) * (4 + 3 * s) + nv * (4 + 8 * visc) * s +
                          ne * 4 * s + rk;
  // What the pass that stages its blocks in LDS reads instead: 1/2-byte
  // local slot ids plus the per-block lists of distinct rows and edges and
  // the per-vertex bases.
  const auto& g = c->stage;
  const bool staged = g.idx_bytes != 0;
  I.stage_idx_bytes = staged ? g.idx_bytes : 0;
  I.stage_max_rows = staged ? g.max_rows : 0;
  I.stage_max_edges = staged ? g.max_edges : 0;
  I.bytes_vertex_staged =
      staged ? I.bytes_vertex_launch -
                   (4.0 - g.idx_bytes) * double(I.n_vslots + I.n_eslots) +
                   double(g.list_ints) * 4
             : 0.0;
}

template <class T>
hfd_status alloc_bufs(hfd_ctx* c, hfd_ctx::Bufs<T>& B, int64_t nv, int64_t ne) {
  hfd_status s;
  for (int k = 0; k < 3; ++k)
    if ((s = dalloc(c, &B.Gv[k], nv)) || (s = dalloc(c, &B.Gg[k], 2 * nv))) return s;
  return dalloc(c, &B.H, ne);
}

hfd_status ensure_mixed_buffers(hfd_ctx* c) {
  hfd_status s;
  const hfd::HostSetup& h = c->hs;
  const int64_t ne = h.ne, nv = h.nv, nvs = h.vptr[h.n_owned], nes = h.eptr[h.n_owned];
  if (!c->fw5) {
    if ((s = dalloc(c, &c->fn, 2 * ne)) || (s = dalloc(c, &c->fw5, 30 * ne)) ||
        (s = dalloc(c, &c->fw3, 18 * ne)) || (s = dalloc(c, &c->fdv, 6 * nvs)) ||
        (s = dalloc(c, &c->fde, 3 * nes)))
      return s;
    if (c->dvis && (s = dalloc(c, &c->fdvis, 5 * nvs))) return s;
    if ((s = alloc_bufs(c, c->b32, nv, ne))) return s;
  }
  HIPCHK(c, hfd::launch_cast(2 * ne, c->n, c->fn, nullptr));
  HIPCHK(c, hfd::launch_cast(30 * ne, c->w5, c->fw5, nullptr));
  HIPCHK(c, hfd::launch_cast(18 * ne, c->w3, c->fw3, nullptr));
  HIPCHK(c, hfd::launch_cast(6 * nvs, c->dv, c->fdv, nullptr));
  HIPCHK(c, hfd::launch_cast(3 * nes, c->de, c->fde, nullptr));
  if (c->dvis) HIPCHK(c, hfd::launch_cast(5 * nvs, c->dvis, c->fdvis, nullptr));
  HIPCHK(c, hipDeviceSynchronize());
  return HFD_OK;
}

hfd::EdgeCoef<double> ecoef64(const hfd_ctx* c) {
  return {c->stg, c->n, c->w5, c->w3, c->erp, c->erow, c->epos, c->e_max_rows};
}
hfd::EdgeCoef<float> ecoef32(const hfd_ctx* c) {
  return {c->stg, c->fn, c->fw5, c->fw3, c->erp, c->erow, c->epos, c->e_max_rows};
}
hfd::VertexCoef<double> vcoef64(const hfd_ctx* c) {
  const auto& g = c->stage;
  return {c->vptr, c->eptr, c->vg,   c->ve,   c->dv,        c->de,       c->dvis,
          c->hrp,  c->hrow, c->hep,  c->hedge, c->lbase,    c->vloc,     c->eloc,
          g.idx_bytes,
          g.max_rows, g.max_edges};
}
hfd::VertexCoef<float> vcoef32(const hfd_ctx* c) {
  const auto& g = c->stage;
  return {c->vptr, c->eptr, c->vg,   c->ve,   c->fdv,       c->fde,      c->fdvis,
          c->hrp,  c->hrow, c->hep,  c->hedge, c->lbase,    c->vloc,     c->eloc,
          g.idx_bytes,
          g.max_rows, g.max_edges};
}

// Device address of `scratch` on the context's device, taken once per device
// with that device current and kept for every later context on it.
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;

hfd_status scratch_setup(hfd_ctx* c) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (c->device >= int(g_scratch_dev.size())) g_scratch_dev.resize(c->device + 1, nullptr);
  if (!g_scratch_dev[c->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, HFD_E_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[c->device] = static_cast<double*>(p);
  }
  c->scratch_dev = g_scratch_dev[c->device];
  return HFD_OK;
}

hfd_status need_device(const hfd_ctx* c) {
  if (!c) return HFD_E_INVAL;
  if (c->device < 0) return fail(const_cast<hfd_ctx*>(c), HFD_E_STATE, "host-only context");
  return HFD_OK;
}

// Brackets one launch with events when timing is on (kind 0 edge, 1 vertex).
struct PassTimer {
  hfd_ctx* c;
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  static hipEvent_t take(hfd_ctx* c) {
    if (!c->ev_pool.empty()) {
      hipEvent_t e = c->ev_pool.back();
      c->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  PassTimer(hfd_ctx* c_, int k, hipStream_t s) : c(c_), kind(k), st(s) {
    if (!c->timing) return;
    a = take(c);
    b = take(c);
    if (a && b && hipEventRecord(a, st) != hipSuccess) a = nullptr;
  }
  ~PassTimer() {
    if (!c->timing || !a || !b) return;
    if (hipEventRecord(b, st) == hipSuccess) c->ev_pending[kind].emplace_back(a, b);
  }
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// One Runge-Kutta step.  `gathered`: B.Gv[0], B.Gg[0] already hold U in
// gather layout (the previous step of hfd_rk_steps wrote it); `carry`: the
// last stage also writes the new state's gather copy there.  The gather rows
// of copying ghosts are never read (every gather is resolved to its source),
// so the carried copy needs no ghost refresh.
template <class T>
hfd_status rk_step_t(hfd_ctx* c, hfd_ctx::Bufs<T>& B, const hfd::EdgeCoef<T>& ec,
                     const hfd::VertexCoef<T>& vc, bool mx, double* U, double dt,
                     const double* dt_dev, hipStream_t st, double* S1 = nullptr,
                     double* S2 = nullptr, bool gathered = false, bool carry = false) {
  // S1, S2: where the two intermediate stages go (work buffers by default)
  if (!S1) S1 = c->U1;
  if (!S2) S2 = c->U2;
  const hfd::HostSetup& h = c->hs;
  const int64_t nv = h.nv, ne = h.ne, no = h.n_owned;
  const GasParams gp = gas_params(c, mx);
  const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
  const int64_t nd = int64_t(h.dir_rows.size());
  if (!gathered) {
    HIPCHK(c, hfd::launch_to_gather<T>(nv, U, gp, B.Gv[0], B.Gg[0], st));
    for (int k = 1; k < 3; ++k)
      HIPCHK(c, hfd::launch_copy_gather_rows<T>(nd, c->dir_rows, B.Gv[0], B.Gg[0], B.Gv[k],
                                                B.Gg[k], st));
  }
  const double* in[3] = {U, S1, S2};
  double* outp[3] = {S1, S2, U};
  for (int k = 0; k < 3; ++k) {
    {
      PassTimer t(c, 0, st);
      HIPCHK(c, hfd::launch_edge<T>(ne, ec, gp, B.Gv[k], B.Gg[k], c->force, B.H, nullptr,
                                    nullptr, nullptr, st));
    }
    hfd::RkArgs rk{U, in[k], outp[k], a[k], b[k], dt, dt_dev};
    PassTimer t(c, 1, st);
    HIPCHK(c, hfd::launch_vertex<T>(no, nv, vc, gp, B.Gv[k], B.Gg[k], B.H, 1, nullptr, rk,
                                    k < 2 ? B.Gv[k + 1] : (carry ? B.Gv[0] : nullptr),
                                    k < 2 ? B.Gg[k + 1] : (carry ? B.Gg[0] : nullptr),
                                    c->flag, st));
  }
  const int64_t ncp = int64_t(h.copy_rows.size());
  HIPCHK(c, hfd::launch_copy_rows<double>(ncp, c->copy_rows, c->copy_src, nv, U, U, st));
  return HFD_OK;
}

hfd_status rk_step_impl(hfd_ctx* c, double* U, double dt, const double* dt_dev,
                        hipStream_t st) {
  if (mixed(c)) return rk_step_t<float>(c, c->b32, ecoef32(c), vcoef32(c), true, U, dt, dt_dev, st);
  return rk_step_t<double>(c, c->b64, ecoef64(c), vcoef64(c), false, U, dt, dt_dev, st);
}

// nsteps x (time step on the device, then a Runge-Kutta step); dt of step i
// into dt_dev[i].
template <class T>
hfd_status rk_steps_t(hfd_ctx* c, hfd_ctx::Bufs<T>& B, const hfd::EdgeCoef<T>& ec,
                      const hfd::VertexCoef<T>& vc, bool mx, double* U, int64_t nsteps,
                      double cfl, double* dt_dev, hipStream_t st) {
  const hfd::HostSetup& h = c->hs;
  hfd_status s;
  for (int64_t i = 0; i < nsteps; ++i) {
    HIPCHK(c, hfd::launch_stable_dt(h.n_owned, h.nv, U, c->hmin, c->o.gamma, cfl, c->dtpart,
                                    c->ndtpart, dt_dev + i, st));
    if ((s = rk_step_t<T>(c, B, ec, vc, mx, U, 0.0, dt_dev + i, st, nullptr, nullptr, i > 0,
                          i + 1 < nsteps)))
      return s;
  }
  return HFD_OK;
}

template <class T>
hfd_status residual_t(hfd_ctx* c, hfd_ctx::Bufs<T>& B, const hfd::EdgeCoef<T>& ec,
                      const hfd::VertexCoef<T>& vc, bool mx, const double* U, double* dU,
                      hipStream_t st) {
  const hfd::HostSetup& h = c->hs;
  const GasParams gp = gas_params(c, mx);
  HIPCHK(c, hfd::launch_to_gather<T>(h.nv, U, gp, B.Gv[0], B.Gg[0], st));
  {
    PassTimer t(c, 0, st);
    HIPCHK(c, hfd::launch_edge<T>(h.ne, ec, gp, B.Gv[0], B.Gg[0], c->force, B.H, nullptr,
                                  nullptr, nullptr, st));
  }
  hfd::RkArgs none{};
  {
    PassTimer t(c, 1, st);
    HIPCHK(c, hfd::launch_vertex<T>(h.n_owned, h.nv, vc, gp, B.Gv[0], B.Gg[0], B.H, 0, dU,
                                    none, nullptr, nullptr, c->flag, st));
  }
  HIPCHK(c, hfd::launch_zero_ghost_rows(h.n_owned, h.nv, dU, st));
  return HFD_OK;
}

template <class T>
hfd_status edge_states_t(hfd_ctx* c, hfd_ctx::Bufs<T>& B, const hfd::EdgeCoef<T>& ec,
                         bool mx, const double* U, double* wlr, double* grad, uint8_t* mask,
                         double* hout, hipStream_t st) {
  const hfd::HostSetup& h = c->hs;
  const GasParams gp = gas_params(c, mx);
  // the derivatives take the branches the edge pass records
  uint8_t* m = mask ? mask : (grad ? c->gmask : nullptr);
  HIPCHK(c, hfd::launch_to_gather<T>(h.nv, U, gp, B.Gv[0], B.Gg[0], st));
  HIPCHK(c, hfd::launch_edge<T>(h.ne, ec, gp, B.Gv[0], B.Gg[0], c->force, B.H, hout, wlr,
                                m, st));
  if (grad)
    HIPCHK(c, hfd::launch_edge_grad<T>(h.ne, ec, c->w5g, c->w3g, gp, B.Gv[0], B.Gg[0], m, grad,
                                       st));
  return HFD_OK;
}


// Transposed maps of the adjoint, by counting sort (deterministic order:
// owner vertex, then slot).
template <class A>
void transpose(int64_t nrows, const std::vector<int32_t, A>& key, std::vector<int32_t>& ptr,
               std::vector<int32_t>& pos) {
  ptr.assign(nrows + 1, 0);
  for (int32_t k : key) ptr[k + 1]++;
  for (int64_t r = 0; r < nrows; ++r) ptr[r + 1] += ptr[r];
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  pos.resize(key.size());
  for (size_t i = 0; i < key.size(); ++i) pos[fill[key[i]]++] = int32_t(i);
}

// Coefficient rows in the order of the transposed maps (rebuilt after an
// import of weights).
hfd_status ensure_adjoint_coefs(hfd_ctx* c) {
  if (c->adj_coef_ready) return HFD_OK;
  const int64_t nes = c->info.n_eslots, nvs = c->info.n_vslots;
  hfd_status s;
  if (!c->de_t && ((s = dalloc(c, &c->de_t, 3 * nes)) || (s = dalloc(c, &c->dv_t, 6 * nvs)) ||
                    (c->dvis && (s = dalloc(c, &c->dvis_t, 5 * nvs)))))
    return s;
  HIPCHK(c, hfd::launch_take_rows(nes, 3, c->ets, c->de, c->de_t, nullptr));
  HIPCHK(c, hfd::launch_take_rows(nvs, 6, c->vts, c->dv, c->dv_t, nullptr));
  if (c->dvis) HIPCHK(c, hfd::launch_take_rows(nvs, 5, c->vts, c->dvis, c->dvis_t, nullptr));
  HIPCHK(c, hipStreamSynchronize(nullptr));
  c->adj_coef_ready = true;
  c->adj_coef32_ready = false;
  return HFD_OK;
}

// Staging lists of the edge reverse: per block of eb consecutive edges
// (entries ptr[e] .. ptr[e+1] of edge e, vertex tv[k]) the sorted distinct
// vertices of its lambda_h entries, and per entry its position in its
// block's list.  Empty when a list is longer than maxrows.
bool adj_stage_lists(int64_t ne, int64_t eb, int maxrows, const std::vector<int32_t>& ptr,
                     const std::vector<int32_t>& tv, std::vector<int32_t>& rp,
                     std::vector<int32_t>& rows, std::vector<uint16_t>& pos) {
  const int64_t nb = (ne + eb - 1) / eb;
  std::vector<std::vector<int32_t>> bl;
  bl.resize(size_t(nb));
  pos.assign(tv.size(), 0);
  int tl[16] = {0};
  hfd::parallel_for(nb, [&](int64_t b0, int64_t b1, unsigned t) {
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t k0 = ptr[b * eb], k1 = ptr[std::min(ne, (b + 1) * eb)];
      std::vector<int32_t>& L = bl[size_t(b)];
      L.assign(tv.begin() + k0, tv.begin() + k1);
      std::sort(L.begin(), L.end());
      L.erase(std::unique(L.begin(), L.end()), L.end());
      if (int64_t(L.size()) > maxrows) {
        tl[t] = std::max(tl[t], int(L.size()));
        continue;
      }
      for (int64_t k = k0; k < k1; ++k)
        pos[size_t(k)] = uint16_t(std::lower_bound(L.begin(), L.end(), tv[k]) - L.begin());
      tl[t] = std::max(tl[t], int(L.size()));
    }
  });
  if (*std::max_element(tl, tl + 16) > maxrows) {
    rp.clear();
    rows.clear();
    pos.clear();
    return false;
  }
  rp.assign(size_t(nb + 1), 0);
  for (int64_t b = 0; b < nb; ++b) rp[b + 1] = rp[b] + int32_t(bl[b].size());
  rows.resize(size_t(rp[nb]));
  for (int64_t b = 0; b < nb; ++b) std::copy(bl[b].begin(), bl[b].end(), rows.begin() + rp[b]);
  return true;
}

hfd_status ensure_adjoint(hfd_ctx* c) {
  if (c->adj_ready) return ensure_adjoint_coefs(c);
  const hfd::HostSetup& h = c->hs;
  const int64_t ne = h.ne, nv = h.nv, no = h.n_owned;
  hfd_status s;
  std::vector<int32_t> ptr, pos;
  // edge <- (owner, edge slot)
  {
    std::vector<int32_t> owner(h.v_edges.size());
    for (int64_t v = 0; v < no; ++v)
      for (int64_t k = h.eptr[v]; k < h.eptr[v + 1]; ++k) owner[k] = int32_t(v);
    transpose(ne, h.v_edges, ptr, pos);
    std::vector<int32_t> tv(pos.size()), ts(pos.size());
    for (size_t i = 0; i < pos.size(); ++i) {
      ts[i] = pos[i];
      tv[i] = owner[pos[i]];
    }
    if ((s = upload(c, &c->etp, ptr)) || (s = upload(c, &c->etv, tv)) || (s = upload(c, &c->ets, ts)))
      return s;
    std::vector<int32_t> rp, rows;
    std::vector<uint16_t> lpos;
    if (!c->o.stage_off && ne > 0 &&
        adj_stage_lists(ne, hfd::kAdjEdgesPerBlock, hfd::kAdjStageRows, ptr, tv, rp, rows, lpos) &&
        ((s = upload(c, &c->alrp, rp)) || (s = upload(c, &c->alrow, rows)) ||
         (s = upload(c, &c->alpos, lpos))))
      return s;
  }
  // gather row <- (owner, vertex slot)
  {
    std::vector<int32_t> owner(h.v_gather.size());
    for (int64_t v = 0; v < no; ++v)
      for (int64_t k = h.vptr[v]; k < h.vptr[v + 1]; ++k) owner[k] = int32_t(v);
    transpose(nv, h.v_gather, ptr, pos);
    std::vector<int32_t> tv(pos.size()), ts(pos.size());
    for (size_t i = 0; i < pos.size(); ++i) {
      ts[i] = pos[i];
      tv[i] = owner[pos[i]];
    }
    if ((s = upload(c, &c->vtp, ptr)) || (s = upload(c, &c->vtv, tv)) || (s = upload(c, &c->vts, ts)))
      return s;
  }
  // gather row <- (edge, stencil position); keys in edge-major order
  {
    std::vector<int32_t> key(6 * ne);
    for (int64_t e = 0; e < ne; ++e)
      for (int j = 0; j < 6; ++j) key[6 * e + j] = h.e_stg[j * ne + e];
    transpose(nv, key, ptr, pos);
    std::vector<int32_t> te(pos.size());
    std::vector<int8_t> tj(pos.size());
    for (size_t i = 0; i < pos.size(); ++i) {
      te[i] = pos[i] / 6;
      tj[i] = int8_t(pos[i] % 6);
    }
    if ((s = upload(c, &c->ntp, ptr)) || (s = upload(c, &c->nte, te)) || (s = upload(c, &c->ntj, tj)))
      return s;
  }
  // copy source -> its ghosts
  {
    std::vector<int32_t> srcs(h.copy_src), order(h.copy_src.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int32_t(i);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return srcs[a] < srcs[b]; });
    std::vector<int32_t> sp{0}, sr, sg;
    for (size_t i = 0; i < order.size(); ++i) {
      const int32_t src = srcs[order[i]];
      if (sr.empty() || sr.back() != src) {
        if (!sr.empty()) sp.push_back(int32_t(i));
        sr.push_back(src);
      }
      sg.push_back(h.copy_rows[order[i]]);
    }
    sp.push_back(int32_t(order.size()));
    if (sr.empty()) sp.assign(1, 0);
    c->n_gsrc = int64_t(sr.size());
    if ((s = upload(c, &c->gsp, sp)) || (s = upload(c, &c->gsr, sr)) || (s = upload(c, &c->gsg, sg)))
      return s;
  }
  if ((s = dalloc(c, &c->bnode, 72 * ne)) || (s = dalloc(c, &c->adj_mask, ne)) ||
      (s = dalloc(c, &c->AL1, 12 * nv)) ||
      (s = dalloc(c, &c->AL2, 12 * nv)) || (s = dalloc(c, &c->AL3, 12 * nv)) ||
      (s = dalloc(c, &c->LGv[0], nv)) || (s = dalloc(c, &c->LGg[0], 2 * nv)) ||
      (s = dalloc(c, &c->LGv[1], nv)) || (s = dalloc(c, &c->LGg[1], 2 * nv)))
    return s;
  c->adj_ready = true;
  return ensure_adjoint_coefs(c);
}

// Buffers and coefficients of one precision.
template <class T> hfd_ctx::Bufs<T>& bufs(hfd_ctx* c);
template <> hfd_ctx::Bufs<double>& bufs<double>(hfd_ctx* c) { return c->b64; }
template <> hfd_ctx::Bufs<float>& bufs<float>(hfd_ctx* c) { return c->b32; }
template <class T> hfd::EdgeCoef<T> ecoef(const hfd_ctx* c);
template <> hfd::EdgeCoef<double> ecoef<double>(const hfd_ctx* c) { return ecoef64(c); }
template <> hfd::EdgeCoef<float> ecoef<float>(const hfd_ctx* c) { return ecoef32(c); }
template <class T> hfd::VertexCoef<T> vcoef(const hfd_ctx* c);
template <> hfd::VertexCoef<double> vcoef<double>(const hfd_ctx* c) { return vcoef64(c); }
template <> hfd::VertexCoef<float> vcoef<float>(const hfd_ctx* c) { return vcoef32(c); }

// The float32 adjoint's buffers and coefficient copies (first use in the
// mixed form; the copies follow the float64 ones).
hfd_status ensure_adjoint32(hfd_ctx* c) {
  hfd_status s;
  if ((s = ensure_adjoint(c))) return s;
  const int64_t ne = c->hs.ne, nv = c->hs.nv;
  const int64_t nes = c->info.n_eslots, nvs = c->info.n_vslots;
  if (!c->fde_t) {
    if ((s = dalloc(c, &c->fde_t, 3 * nes)) || (s = dalloc(c, &c->fdv_t, 6 * nvs)) ||
        (c->dvis_t && (s = dalloc(c, &c->fdvis_t, 5 * nvs))) ||
        (s = dalloc(c, &c->bnode32, 72 * ne)) ||
        (s = dalloc(c, &c->LGv32[0], nv)) || (s = dalloc(c, &c->LGg32[0], 2 * nv)) ||
        (s = dalloc(c, &c->LGv32[1], nv)) || (s = dalloc(c, &c->LGg32[1], 2 * nv)))
      return s;
    c->adj_coef32_ready = false;
  }
  if (!c->adj_coef32_ready) {
    HIPCHK(c, hfd::launch_cast(3 * nes, c->de_t, c->fde_t, nullptr));
    HIPCHK(c, hfd::launch_cast(6 * nvs, c->dv_t, c->fdv_t, nullptr));
    if (c->dvis_t) HIPCHK(c, hfd::launch_cast(5 * nvs, c->dvis_t, c->fdvis_t, nullptr));
    HIPCHK(c, hipStreamSynchronize(nullptr));
    c->adj_coef32_ready = true;
  }
  return HFD_OK;
}

hfd_status ensure_adjoint_t(hfd_ctx* c) { return mixed(c) ? ensure_adjoint32(c) : ensure_adjoint(c); }

// Lambda gather buffer k (0, 1) of the precision.
template <class T> hfd::V4<T>* lam_gv(hfd_ctx* c, int k);
template <> hfd::V4<double>* lam_gv<double>(hfd_ctx* c, int k) { return c->LGv[k]; }
template <> hfd::V4<float>* lam_gv<float>(hfd_ctx* c, int k) { return c->LGv32[k]; }
template <class T> hfd::V4<T>* lam_gg(hfd_ctx* c, int k);
template <> hfd::V4<double>* lam_gg<double>(hfd_ctx* c, int k) { return c->LGg[k]; }
template <> hfd::V4<float>* lam_gg<float>(hfd_ctx* c, int k) { return c->LGg32[k]; }

// out = J(U)^T lam (owned rows; out may be null when rc consumes it), U given
// in both layouts (SoA U, gather Gv/Gg of the precision: in float32 the
// perturbation from w_ref).  lam is read in gather buffer k, converted
// there first when `convert`; rc: the fused Runge-Kutta combination.
template <class T>
hfd_status adjoint_apply(hfd_ctx* c, const double* U, const hfd::V4<T>* Gv,
                         const hfd::V4<T>* Gg, const double* lam, int k, bool convert,
                         double* out, const hfd::AdjCombine<T>& rc, hipStream_t st) {
  constexpr bool f32 = sizeof(T) == 4;
  const hfd::HostSetup& h = c->hs;
  hfd::V4<T>* LGv = lam_gv<T>(c, k);
  hfd::V4<T>* LGg = lam_gg<T>(c, k);
  // lambda in gather layout, no reference state
  if (convert)
    HIPCHK(c, hfd::launch_to_gather<T>(h.nv, lam, gas_params(c, false), LGv, LGg, st));
  hfd::AdjointArgs<T> a{};
  a.ne = h.ne;
  a.nowned = h.n_owned;
  a.nv = h.nv;
  a.etp = c->etp; a.etv = c->etv;
  a.lrp = c->alrp; a.lrow = c->alrow; a.lpos = c->alpos;
  a.Lv = LGv; a.Lg = LGg;
  a.ec = ecoef<T>(c);
  a.gp = gas_params(c, f32);
  a.Gv = Gv; a.Gg = Gg;
  a.force = c->force;
  // The paper switch's decisions are the forward edge pass's at this state:
  // that kernel writes them (its fluxes go to the edge-flux work buffer) and
  // the reverse takes them as a forced mask, so that it differentiates the
  // branches the forward took, also where its own arithmetic would put
  // omega_1 on the other side of a threshold (float32 rounding).
  if (!c->force && c->o.switch_mode == HFD_SWITCH_PAPER) {
    HIPCHK(c, hfd::launch_edge<T>(h.ne, a.ec, a.gp, Gv, Gg, nullptr, bufs<T>(c).H, nullptr,
                                  nullptr, c->adj_mask, st));
    a.force = c->adj_mask;
  }
  a.U = U;
  a.vtp = c->vtp; a.vtv = c->vtv;
  a.ntp = c->ntp; a.nte = c->nte; a.ntj = c->ntj;
  a.out = out;
  a.rc = rc;
  if constexpr (f32) {
    a.de_t = c->fde_t; a.dv_t = c->fdv_t; a.dvis_t = c->fdvis_t;
    a.bnode = c->bnode32;
  } else {
    a.de_t = c->de_t; a.dv_t = c->dv_t; a.dvis_t = c->dvis_t;
    a.bnode = c->bnode;
  }
  HIPCHK(c, hfd::launch_adjoint_residual<T>(a, st));
  if (out) HIPCHK(c, hfd::launch_zero_ghost_rows(h.n_owned, h.nv, out, st));
  return HFD_OK;
}

}  // namespace

extern "C" {

void hfd_default_opts(hfd_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->gamma = 1.4;
  o->gas_R = 1.0;
  o->mu = 0.0;
  o->prandtl = 0.72;
  o->weno_eps = 1e-6;
  o->sw_lo = 0.01;
  o->sw_hi = 0.79;
  o->w3_cap = 0.0;
  o->switch_mode = HFD_SWITCH_PAPER;
  o->precision = HFD_FP64;
  o->order = HFD_ORDER_HILBERT;
  o->deg_inv = HFD_DEFAULT_DEG_INV;
}

const char* hfd_status_string(hfd_status s) {
  switch (s) {
    case HFD_OK: return "ok";
    case HFD_E_INVAL: return "invalid argument";
    case HFD_E_MESH: return "unusable mesh";
    case HFD_E_NOMEM: return "out of memory";
    case HFD_E_DEVICE: return "device error";
    case HFD_E_NUMERIC: return "non-finite or non-physical state";
    case HFD_E_STATE: return "invalid call for this context";
  }
  return "unknown status";
}

const char* hfd_last_error(const hfd_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

hfd_status hfd_destroy(hfd_ctx* ctx) {
  if (!ctx) return HFD_OK;
  if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
  for (int k = 0; k < 2; ++k)
    for (auto& pr : ctx->ev_pending[k]) {
      (void)hipEventSynchronize(pr.second);
      ctx->ev_pool.push_back(pr.first);
      ctx->ev_pool.push_back(pr.second);
    }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (void* p : ctx->allocs) (void)hipFree(p);
  delete ctx;
  return HFD_OK;
}

hfd_status hfd_create(const double* xy, int64_t nv, const int32_t* tri, int64_t nt,
                      const int32_t* ghost_src, const hfd_opts* o, int device,
                      hfd_ctx** out) {
  if (!out) return HFD_E_INVAL;
  *out = nullptr;
  hfd_ctx* c = new (std::nothrow) hfd_ctx();
  if (!c) return HFD_E_NOMEM;
  auto bail = [&](hfd_status s) {
    g_create_err = c->err;
    hfd_destroy(c);
    return s;
  };
  if (o) c->o = *o;
  else hfd_default_opts(&c->o);
  const hfd_opts& op = c->o;
  if (!(op.gamma > 1.0) || op.mu < 0.0 || !(op.weno_eps > 0.0) || op.w3_cap < 0.0 ||
      op.switch_mode < 0 || op.switch_mode > 2 || op.precision < 0 || op.precision > 1 ||
      op.flux < HFD_FLUX_RUSANOV || op.flux > HFD_FLUX_HLLC || op.order < HFD_ORDER_NONE ||
      op.order > HFD_ORDER_RCM || op.edge_grad < 0 || op.edge_grad > 1 ||
      (op.deg_inv != 4 && op.deg_inv != 5) ||
      op.period[0] < 0.0 || op.period[1] < 0.0 ||
      (op.mu > 0.0 && (!(op.prandtl > 0.0) || !(op.gas_R > 0.0)))) {
    c->err = "invalid options";
    return bail(HFD_E_INVAL);
  }
  auto t0 = std::chrono::steady_clock::now();
  hfd_status s = hfd::host_setup(xy, nv, tri, nt, ghost_src, op, &c->hs, &c->err);
  if (s != HFD_OK) return bail(s);
  hfd::HostSetup& h = c->hs;
  hfd_info& I = c->info;
  I.nv = h.nv;
  I.n_owned = h.n_owned;
  I.n_dirichlet = h.n_dir;
  I.n_copy_ghost = h.n_copy;
  I.n_edges_mesh = h.ne_mesh;
  I.n_edges = h.ne;
  I.n_vslots = h.vptr[h.n_owned];
  I.n_eslots = h.eptr[h.n_owned];
  I.max_vslots = h.max_vs;
  I.max_eslots = h.max_es;
  I.setup_ms[0] = ms_since(t0);
  // the passes take the Dirichlet ghosts as the rows right after the owned ones
  for (size_t k = 0; k < h.dir_rows.size(); ++k)
    if (h.dir_rows[k] != h.n_owned + int64_t(k)) {
      c->err = "internal: Dirichlet ghost rows are not contiguous after the owned rows";
      return bail(HFD_E_MESH);
    }
  if (I.n_vslots >= (int64_t(1) << 31) || I.n_eslots >= (int64_t(1) << 31)) {
    c->err = "mesh too large for 32-bit slot offsets";
    return bail(HFD_E_MESH);
  }
  const int64_t msys = 2 * int64_t(h.max_vs) + h.max_es;
  if (msys > 192 || h.max_vs > 64) {
    c->err = "divergence system with " + std::to_string(msys) + " rows (limit 192) or " +
             std::to_string(h.max_vs) + " stencil vertices (limit 64)";
    return bail(HFD_E_MESH);
  }
  build_stage(c);
  byte_model(c);
  if (device < 0) {
    *out = c;
    return HFD_OK;
  }
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    c->err = "hipSetDevice failed";
    return bail(HFD_E_DEVICE);
  }
  if ((s = scratch_setup(c))) return bail(s);
  auto t1 = std::chrono::steady_clock::now();
  const int64_t ne = h.ne, no = h.n_owned, nvs = I.n_vslots, nes = I.n_eslots;
  std::vector<int32_t> vp32(no + 1), ep32(no + 1);
  for (int64_t k = 0; k <= no; ++k) {
    vp32[k] = int32_t(h.vptr[k]);
    ep32[k] = int32_t(h.eptr[k]);
  }
  double *d_pts = nullptr, *d_eh = nullptr, *d_vpts = nullptr, *d_mpts = nullptr,
         *d_vh = nullptr;
  int64_t *d_vptr64 = nullptr, *d_eptr64 = nullptr;
  int32_t* d_status = nullptr;
  if ((s = upload(c, &c->stg, h.e_stg)) || (s = upload(c, &c->n, h.e_n)) ||
      (s = upload(c, &c->vptr, vp32)) || (s = upload(c, &c->eptr, ep32)) ||
      (s = upload(c, &c->vg, h.v_gather)) || (s = upload(c, &c->ve, h.v_edges)) ||
      (s = upload(c, &c->hmin, h.v_hmin)) || (s = upload(c, &c->dir_rows, h.dir_rows)) ||
      (s = upload(c, &c->copy_rows, h.copy_rows)) || (s = upload(c, &c->copy_src, h.copy_src)) ||
      (s = upload(c, &d_pts, h.e_pts)) || (s = upload(c, &d_eh, h.e_h)) ||
      (s = upload(c, &d_vpts, h.v_pts)) || (s = upload(c, &d_mpts, h.m_pts)) ||
      (s = upload(c, &d_vh, h.v_h)) ||
      (s = upload(c, &d_vptr64, h.vptr)) || (s = upload(c, &d_eptr64, h.eptr)))
    return bail(s);
  if (HFD_EDGE_STAGE && !op.stage_off && ne > 0) {
    std::vector<int32_t> erp, erow;
    std::vector<uint16_t> epos;
    edge_stage_lists(h, erp, erow, epos, c->e_max_rows);
    if (!erp.empty() && ((s = upload(c, &c->erp, erp)) || (s = upload(c, &c->erow, erow)) ||
                         (s = upload(c, &c->epos, epos))))
      return bail(s);
  }
  if (c->stage.idx_bytes) {
    auto& g = c->stage;
    if ((s = upload(c, &c->hrp, g.rp)) || (s = upload(c, &c->hrow, g.rows)) ||
        (s = upload(c, &c->hep, g.ep)) || (s = upload(c, &c->hedge, g.edges)) ||
        (s = upload(c, &c->lbase, g.base)))
      return bail(s);
    if (g.idx_bytes == 1) {
      std::vector<uint8_t> v8(g.vloc.begin(), g.vloc.end()), e8(g.eloc.begin(), g.eloc.end());
      uint8_t *pv = nullptr, *pe = nullptr;
      if ((s = upload(c, &pv, v8)) || (s = upload(c, &pe, e8))) return bail(s);
      c->vloc = pv;
      c->eloc = pe;
    } else {
      uint16_t *pv = nullptr, *pe = nullptr;
      if ((s = upload(c, &pv, g.vloc)) || (s = upload(c, &pe, g.eloc))) return bail(s);
      c->vloc = pv;
      c->eloc = pe;
    }
    // the host copies are not needed any more (the byte model keeps list_ints)
    std::vector<int32_t>().swap(g.rp);
    std::vector<int32_t>().swap(g.rows);
    std::vector<int32_t>().swap(g.ep);
    std::vector<int32_t>().swap(g.edges);
    std::vector<uint32_t>().swap(g.base);
    std::vector<uint16_t>().swap(g.vloc);
    std::vector<uint16_t>().swap(g.eloc);
  }
  if ((s = dalloc(c, &c->w5, 30 * ne)) || (s = dalloc(c, &c->w3, 18 * ne)) ||
      (s = dalloc(c, &c->rank, 2 * ne)) || (s = dalloc(c, &c->trunc3, 6 * ne)) ||
      (s = dalloc(c, &c->dv, 6 * nvs)) || (s = dalloc(c, &c->de, 3 * nes)) ||
      (s = dalloc(c, &d_status, no)) || (s = dalloc(c, &c->U1, 12 * h.nv)) ||
      (s = dalloc(c, &c->U2, 12 * h.nv)) || (s = alloc_bufs(c, c->b64, h.nv, ne)) ||
      (s = dalloc(c, &c->flag, 1)))
    return bail(s);
  if (op.mu > 0.0 && (s = dalloc(c, &c->dvis, 5 * nvs))) return bail(s);
  if (op.edge_grad && ((s = dalloc(c, &c->w5g, 60 * ne)) || (s = dalloc(c, &c->w3g, 36 * ne)) ||
                       (s = dalloc(c, &c->gmask, ne))))
    return bail(s);
  c->ndtpart = std::max<int64_t>(1, std::min<int64_t>(1024, (no + 255) / 256));
  if ((s = dalloc(c, &c->dtpart, c->ndtpart))) return bail(s);
  if (hipMemset(c->flag, 0, sizeof(int32_t)) != hipSuccess) {
    c->err = "hipMemset failed";
    return bail(HFD_E_DEVICE);
  }
  I.setup_ms[1] = ms_since(t1);
  auto t2 = std::chrono::steady_clock::now();
  // ---- precompute ----------------------------------------------------------
  hipError_t he;
  if ((he = hfd::launch_edge_weights(ne, d_pts, d_eh, op.w3_cap, c->w5, c->w3, c->rank,
                                     c->trunc3, c->w5g, c->w3g, nullptr)) != hipSuccess ||
      (he = hfd::launch_div_rows(no, int(msys), op.deg_inv, d_vptr64, d_eptr64, d_vpts, d_mpts, c->ve, c->n,
                                 ne, d_vh, c->dv, c->de, d_status, nullptr)) != hipSuccess ||
      (he = hipDeviceSynchronize()) != hipSuccess) {
    c->err = std::string("precompute: ") + hipGetErrorString(he);
    return bail(HFD_E_DEVICE);
  }
  std::vector<int32_t> stat(no);
  if (hipMemcpy(stat.data(), d_status, no * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
    c->err = "status copy failed";
    return bail(HFD_E_DEVICE);
  }
  for (int64_t k = 0; k < no; ++k)
    if (stat[k] == 1) {
      c->err = "rank-deficient divergence system at vertex " +
               std::to_string(h.old_of_new[k]);
      return bail(HFD_E_MESH);
    }
  if (op.mu > 0.0) {
    if ((he = hfd::launch_visc_rows(no, d_vptr64, d_vpts, d_vh, c->dvis, d_status,
                                    nullptr)) != hipSuccess ||
        (he = hipDeviceSynchronize()) != hipSuccess) {
      c->err = std::string("viscous precompute: ") + hipGetErrorString(he);
      return bail(HFD_E_DEVICE);
    }
  }
  {
    std::vector<int32_t> rk(2 * ne);
    std::vector<int8_t> t3(6 * ne);
    if (hipMemcpy(rk.data(), c->rank, rk.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(t3.data(), c->trunc3, t3.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      c->err = "rank copy failed";
      return bail(HFD_E_DEVICE);
    }
    for (int32_t r : rk) I.rank_hist[std::min(15, std::max(0, r))]++;
    for (int8_t t : t3) I.w3_truncated += (t > 0);
  }
  for (void* p : {(void*)d_pts, (void*)d_eh, (void*)d_vpts, (void*)d_mpts,
                  (void*)d_vh, (void*)d_vptr64, (void*)d_eptr64, (void*)d_status})
    dfree(c, p);
  // host copies of the frames are no longer needed
  hfd::HostArray<double>().swap(h.e_pts);
  hfd::HostArray<double>().swap(h.v_pts);
  hfd::HostArray<double>().swap(h.m_pts);
  I.setup_ms[2] = ms_since(t2);
  if (mixed(c) && (s = ensure_mixed_buffers(c))) return bail(s);
  I.setup_ms[3] = ms_since(t0);
  *out = c;
  return HFD_OK;
}

hfd_status hfd_get_info(const hfd_ctx* ctx, hfd_info* out) {
  if (!ctx || !out) return HFD_E_INVAL;
  *out = ctx->info;
  return HFD_OK;
}

hfd_status hfd_permutation(const hfd_ctx* ctx, int32_t* new_of_old) {
  if (!ctx || !new_of_old) return HFD_E_INVAL;
  std::memcpy(new_of_old, ctx->hs.new_of_old.data(), ctx->hs.nv * sizeof(int32_t));
  return HFD_OK;
}

hfd_status hfd_export_edges(const hfd_ctx* ctx, int32_t* ends, int32_t* stencil) {
  if (!ctx) return HFD_E_INVAL;
  if (ends) std::memcpy(ends, ctx->hs.e_end.data(), ctx->hs.e_end.size() * 4);
  if (stencil) std::memcpy(stencil, ctx->hs.e_st.data(), ctx->hs.e_st.size() * 4);
  return HFD_OK;
}

hfd_status hfd_export_vertex_stencils(const hfd_ctx* ctx, int64_t* vptr, int32_t* vnodes,
                                      int64_t* eptr, int32_t* vedges) {
  if (!ctx) return HFD_E_INVAL;
  const hfd::HostSetup& h = ctx->hs;
  if (vptr) std::memcpy(vptr, h.vptr.data(), h.vptr.size() * 8);
  if (eptr) std::memcpy(eptr, h.eptr.data(), h.eptr.size() * 8);
  if (vnodes) std::memcpy(vnodes, h.v_nodes.data(), h.v_nodes.size() * 4);
  if (vedges) std::memcpy(vedges, h.v_edges.data(), h.v_edges.size() * 4);
  return HFD_OK;
}

hfd_status hfd_export_weights(const hfd_ctx* ctx, double* w5, double* w3, int32_t* rank,
                              double* dv, double* de, double* dvis) {
  hfd_status s = need_device(ctx);
  if (s) return s;
  hfd_ctx* c = const_cast<hfd_ctx*>(ctx);
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  const int64_t ne = c->hs.ne;
  // device records [2 sides][ne][n] -> [ne][2 sides][n]
  auto records_to_host = [&](const double* d, int64_t n, double* out) -> hfd_status {
    std::vector<double> tmp(2 * n * ne);
    HIPCHK(c, hipMemcpy(tmp.data(), d, tmp.size() * 8, hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < ne; ++e)
      for (int64_t sd = 0; sd < 2; ++sd)
        for (int64_t k = 0; k < n; ++k) out[(e * 2 + sd) * n + k] = tmp[(sd * ne + e) * n + k];
    return HFD_OK;
  };
  if (w5 && (s = records_to_host(c->w5, 15, w5))) return s;
  if (w3 && (s = records_to_host(c->w3, 9, w3))) return s;
  if (rank) {
    std::vector<int32_t> tmp(2 * ne);
    HIPCHK(c, hipMemcpy(tmp.data(), c->rank, tmp.size() * 4, hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < ne; ++e)
      for (int r = 0; r < 2; ++r) rank[2 * e + r] = tmp[r * ne + e];
  }
  if (dv) HIPCHK(c, hipMemcpy(dv, c->dv, 6 * c->info.n_vslots * 8, hipMemcpyDeviceToHost));
  if (de) HIPCHK(c, hipMemcpy(de, c->de, 3 * c->info.n_eslots * 8, hipMemcpyDeviceToHost));
  if (dvis) {
    if (!c->dvis) return fail(c, HFD_E_STATE, "no viscous rows (mu == 0)");
    HIPCHK(c, hipMemcpy(dvis, c->dvis, 5 * c->info.n_vslots * 8, hipMemcpyDeviceToHost));
  }
  return HFD_OK;
}

hfd_status hfd_import_weights(hfd_ctx* c, const double* w5, const double* w3,
                              const double* dv, const double* de, const double* dvis) {
  hfd_status s = need_device(c);
  if (s) return s;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  const int64_t ne = c->hs.ne;
  // [ne][2 sides][n] -> device records [2 sides][ne][n]
  auto host_to_records = [&](const double* in, int64_t n, double* d) -> hfd_status {
    std::vector<double> tmp(2 * n * ne);
    for (int64_t e = 0; e < ne; ++e)
      for (int64_t sd = 0; sd < 2; ++sd)
        for (int64_t k = 0; k < n; ++k) tmp[(sd * ne + e) * n + k] = in[(e * 2 + sd) * n + k];
    HIPCHK(c, hipMemcpy(d, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice));
    return HFD_OK;
  };
  if (w5 && (s = host_to_records(w5, 15, c->w5))) return s;
  if (w3 && (s = host_to_records(w3, 9, c->w3))) return s;
  if (dv) HIPCHK(c, hipMemcpy(c->dv, dv, 6 * c->info.n_vslots * 8, hipMemcpyHostToDevice));
  if (de) HIPCHK(c, hipMemcpy(c->de, de, 3 * c->info.n_eslots * 8, hipMemcpyHostToDevice));
  if (dv || de || dvis) c->adj_coef_ready = false;
  if (dvis) {
    if (!c->dvis) return fail(c, HFD_E_STATE, "no viscous rows (mu == 0)");
    HIPCHK(c, hipMemcpy(c->dvis, dvis, 5 * c->info.n_vslots * 8, hipMemcpyHostToDevice));
  }
  if (c->fw5) return ensure_mixed_buffers(c);
  return HFD_OK;
}

hfd_status hfd_export_grad_weights(const hfd_ctx* ctx, double* w5g, double* w3g) {
  hfd_status s = need_device(ctx);
  if (s) return s;
  hfd_ctx* c = const_cast<hfd_ctx*>(ctx);
  if (!c->w5g) return fail(c, HFD_E_STATE, "context created without hfd_opts.edge_grad");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  const int64_t ne = c->hs.ne;
  for (auto [d, rows, out] : {std::tuple<const double*, int64_t, double*>{c->w5g, 60, w5g},
                              std::tuple<const double*, int64_t, double*>{c->w3g, 36, w3g}}) {
    if (!out) continue;
    std::vector<double> tmp(rows * ne);
    HIPCHK(c, hipMemcpy(tmp.data(), d, tmp.size() * 8, hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < ne; ++e)
      for (int64_t r = 0; r < rows; ++r) out[e * rows + r] = tmp[r * ne + e];
  }
  return HFD_OK;
}

hfd_status hfd_import_grad_weights(hfd_ctx* c, const double* w5g, const double* w3g) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!c->w5g) return fail(c, HFD_E_STATE, "context created without hfd_opts.edge_grad");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  const int64_t ne = c->hs.ne;
  for (auto [in, rows, d] : {std::tuple<const double*, int64_t, double*>{w5g, 60, c->w5g},
                             std::tuple<const double*, int64_t, double*>{w3g, 36, c->w3g}}) {
    if (!in) continue;
    std::vector<double> tmp(rows * ne);
    for (int64_t e = 0; e < ne; ++e)
      for (int64_t r = 0; r < rows; ++r) tmp[r * ne + e] = in[e * rows + r];
    HIPCHK(c, hipMemcpy(d, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice));
  }
  return HFD_OK;
}

hfd_status hfd_set_precision(hfd_ctx* c, int32_t precision, const double* w_ref) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (precision != HFD_FP64 && precision != HFD_FP32_MIXED)
    return fail(c, HFD_E_INVAL, "precision must be HFD_FP64 or HFD_FP32_MIXED");
  HIPCHK(c, hipSetDevice(c->device));
  if (w_ref)
    for (int q = 0; q < 4; ++q) c->o.w_ref[q] = w_ref[q];
  c->o.precision = precision;
  byte_model(c);
  if (precision == HFD_FP32_MIXED) return ensure_mixed_buffers(c);
  return HFD_OK;
}

hfd_status hfd_set_flux(hfd_ctx* c, int32_t flux) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (flux < HFD_FLUX_RUSANOV || flux > HFD_FLUX_HLLC)
    return fail(c, HFD_E_INVAL, "flux must be HFD_FLUX_RUSANOV, HFD_FLUX_ROE or HFD_FLUX_HLLC");
  c->o.flux = flux;
  return HFD_OK;
}

hfd_status hfd_residual(hfd_ctx* c, const double* U, double* dU, void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !dU) return fail(c, HFD_E_INVAL, "null state");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (mixed(c)) return residual_t<float>(c, c->b32, ecoef32(c), vcoef32(c), true, U, dU, st);
  return residual_t<double>(c, c->b64, ecoef64(c), vcoef64(c), false, U, dU, st);
}

hfd_status hfd_rk_step(hfd_ctx* c, double* U, double dt, void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U) return fail(c, HFD_E_INVAL, "null state");
  return rk_step_impl(c, U, dt, nullptr, static_cast<hipStream_t>(stream));
}

hfd_status hfd_rk_step_dev(hfd_ctx* c, double* U, const double* dt_dev, void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !dt_dev) return fail(c, HFD_E_INVAL, "null state or dt");
  return rk_step_impl(c, U, 0.0, dt_dev, static_cast<hipStream_t>(stream));
}

hfd_status hfd_rk_steps(hfd_ctx* c, double* U, int64_t nsteps, double cfl, double* dt_dev,
                        void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !dt_dev || nsteps < 0 || !(cfl > 0.0))
    return fail(c, HFD_E_INVAL, "null pointer, nsteps < 0 or cfl <= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (mixed(c)) return rk_steps_t<float>(c, c->b32, ecoef32(c), vcoef32(c), true, U, nsteps, cfl, dt_dev, st);
  return rk_steps_t<double>(c, c->b64, ecoef64(c), vcoef64(c), false, U, nsteps, cfl, dt_dev, st);
}

hfd_status hfd_stable_dt(hfd_ctx* c, const double* U, double cfl, double* dt_dev,
                         void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !dt_dev || !(cfl > 0.0)) return fail(c, HFD_E_INVAL, "null pointer or cfl <= 0");
  HIPCHK(c, hfd::launch_stable_dt(c->hs.n_owned, c->hs.nv, U, c->hmin, c->o.gamma, cfl,
                                  c->dtpart, c->ndtpart, dt_dev,
                                  static_cast<hipStream_t>(stream)));
  return HFD_OK;
}

hfd_status hfd_stable_dt_noalloc(hfd_ctx* c, const double* U, double cfl, double* dt_dev,
                                 void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !dt_dev || !(cfl > 0.0)) return fail(c, HFD_E_INVAL, "null pointer or cfl <= 0");
  if (!c->scratch_dev) return fail(c, HFD_E_STATE, "scratch address not set up");
  // one partial minimum per 256 owned vertices, all in the shared scratch
  const int64_t np = std::max<int64_t>(1, (c->hs.n_owned + 255) / 256);
  if (np > kNoallocDtPartials)
    return fail(c, HFD_E_INVAL,
                "hfd_stable_dt_noalloc: " + std::to_string(c->hs.n_owned) +
                    " owned vertices, more than the " +
                    std::to_string(kNoallocDtPartials * 256) +
                    " its scratch covers (use hfd_stable_dt)");
  HIPCHK(c, hfd::launch_stable_dt(c->hs.n_owned, c->hs.nv, U, c->hmin, c->o.gamma, cfl,
                                  c->scratch_dev, np, dt_dev,
                                  static_cast<hipStream_t>(stream)));
  return HFD_OK;
}

hfd_status hfd_edge_states(hfd_ctx* c, const double* U, double* wlr, double* grad,
                           uint8_t* mask, double* hout, void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !wlr) return fail(c, HFD_E_INVAL, "null state or output");
  if (grad && !c->w5g)
    return fail(c, HFD_E_STATE,
                "midpoint derivatives need a context created with hfd_opts.edge_grad = 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (mixed(c))
    return edge_states_t<float>(c, c->b32, ecoef32(c), true, U, wlr, grad, mask, hout, st);
  return edge_states_t<double>(c, c->b64, ecoef64(c), false, U, wlr, grad, mask, hout, st);
}

hfd_status hfd_force_switch_mask(hfd_ctx* c, const uint8_t* mask_dev) {
  hfd_status s = need_device(c);
  if (s) return s;
  c->force = mask_dev;
  return HFD_OK;
}

hfd_status hfd_fill_ghosts(hfd_ctx* c, double* U, void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U) return fail(c, HFD_E_INVAL, "null state");
  const int64_t ncp = int64_t(c->hs.copy_rows.size());
  HIPCHK(c, hfd::launch_copy_rows<double>(ncp, c->copy_rows, c->copy_src, c->hs.nv, U, U,
                                          static_cast<hipStream_t>(stream)));
  return HFD_OK;
}

hfd_status hfd_check(hfd_ctx* c, void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(c, hipStreamSynchronize(st));
  int32_t f = 0;
  HIPCHK(c, hipMemcpy(&f, c->flag, sizeof(f), hipMemcpyDeviceToHost));
  if (f) {
    HIPCHK(c, hipMemset(c->flag, 0, sizeof(int32_t)));
    return fail(c, HFD_E_NUMERIC, "non-finite value or rho <= 0 or p <= 0 at an owned vertex");
  }
  return HFD_OK;
}


hfd_status hfd_adjoint_residual(hfd_ctx* c, const double* U, const double* lam, double* out,
                                void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !lam || !out) return fail(c, HFD_E_INVAL, "null pointer");
  if ((s = ensure_adjoint_t(c))) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nv = c->hs.nv;
  if (mixed(c)) {
    auto& B = c->b32;
    HIPCHK(c, hfd::launch_to_gather<float>(nv, U, gas_params(c, true), B.Gv[0], B.Gg[0], st));
    return adjoint_apply<float>(c, U, B.Gv[0], B.Gg[0], lam, 0, true, out, {}, st);
  }
  auto& B = c->b64;
  HIPCHK(c, hfd::launch_to_gather<double>(nv, U, gas_params(c, false), B.Gv[0], B.Gg[0], st));
  return adjoint_apply<double>(c, U, B.Gv[0], B.Gg[0], lam, 0, true, out, {}, st);
}

extern "C++" {
namespace {

// Adjoint of one RK3 step from U with stages U1, U2 (recomputed into the
// work buffers when null), in the context's precision: the stage states in
// its gather layout, the adjoint residuals in its arithmetic, the
// Runge-Kutta combinations of lambda in float64.
template <class T>
hfd_status rk_step_adjoint_t(hfd_ctx* c, const double* U, const double* U1in,
                             const double* U2in, double dt, const double* lam_np1,
                             double* lam_n, hipStream_t st) {
  constexpr bool f32 = sizeof(T) == 4;
  const hfd::HostSetup& h = c->hs;
  const int64_t nv = h.nv, ne = h.ne, no = h.n_owned, n12 = 12 * nv;
  const int64_t nd = int64_t(h.dir_rows.size());
  auto& B = bufs<T>(c);
  const GasParams gp = gas_params(c, f32);
  const double* Us[3] = {U, U1in, U2in};
  if (U1in) {
    // the step's input and the given stages in gather layout, Dirichlet rows
    // from U (internal rows no .. no + nd)
    const hfd::StageGathers<T> g{{B.Gv[0], B.Gv[1], B.Gv[2]}, {B.Gg[0], B.Gg[1], B.Gg[2]}};
    HIPCHK(c, hfd::launch_stage_gathers<T>(nv, no, no + nd, U, U1in, U2in, gp, g, st));
  } else {
    HIPCHK(c, hfd::launch_to_gather<T>(nv, U, gp, B.Gv[0], B.Gg[0], st));
    // forward stages 1 and 2: U1, U2 and their gather copies
    for (int k = 1; k < 3; ++k)
      HIPCHK(c, hfd::launch_copy_gather_rows<T>(nd, c->dir_rows, B.Gv[0], B.Gg[0], B.Gv[k],
                                                B.Gg[k], st));
    HIPCHK(c, hfd::launch_copy_rows<double>(nd, c->dir_rows, nullptr, nv, U, c->U1, st));
    HIPCHK(c, hfd::launch_copy_rows<double>(nd, c->dir_rows, nullptr, nv, U, c->U2, st));
    const double a[2] = {0.0, 0.75}, b[2] = {1.0, 0.25};
    const double* in[2] = {U, c->U1};
    double* outp[2] = {c->U1, c->U2};
    for (int k = 0; k < 2; ++k) {
      HIPCHK(c, hfd::launch_edge<T>(ne, ecoef<T>(c), gp, B.Gv[k], B.Gg[k], c->force, B.H,
                                    nullptr, nullptr, nullptr, st));
      hfd::RkArgs rk{U, in[k], outp[k], a[k], b[k], dt, nullptr};
      HIPCHK(c, hfd::launch_vertex<T>(no, nv, vcoef<T>(c), gp, B.Gv[k], B.Gg[k], B.H, 1,
                                      nullptr, rk, B.Gv[k + 1], B.Gg[k + 1], c->flag, st));
    }
    Us[1] = c->U1;
    Us[2] = c->U2;
  }
  // reverse.  A3 = lam_{n+1} with the final ghost fill transposed (lam_{n+1}
  // itself when there are no copying ghosts).  The combinations of each
  // stage run in the epilogue of its vertex pass (owned rows), which also
  // writes the next stage's lambda in gather layout (the two buffers
  // alternate: a stage reads one while its epilogue writes the other).
  hfd_status s;
  double *L2 = c->AL2, *L1 = c->AL1;
  const double* A3 = lam_np1;
  if (c->n_gsrc > 0) {
    HIPCHK(c, hipMemcpyAsync(c->AL3, lam_np1, n12 * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hfd::launch_adj_copy_ghosts(c->n_gsrc, c->gsp, c->gsr, c->gsg, nv, c->AL3, st));
    A3 = c->AL3;
  }
  // stage 3: U3 = U/3 + 2/3 (U2 + dt R(U2)):
  //   L2 = 2/3 A3 + 2/3 dt J^T A3, lam_n = 1/3 A3
  const hfd::AdjCombine<T> r3{A3, L2, lam_gv<T>(c, 1), lam_gg<T>(c, 1), lam_n,
                              2.0 / 3.0, 2.0 / 3.0 * dt, 0.0, 1.0 / 3.0, 0.0};
  if ((s = adjoint_apply<T>(c, Us[2], B.Gv[2], B.Gg[2], A3, 0, true, nullptr, r3, st))) return s;
  // stage 2: U2 = 3/4 U + 1/4 (U1 + dt R(U1)):
  //   L1 = 1/4 L2 + 1/4 dt J^T L2, lam_n += 3/4 L2
  const hfd::AdjCombine<T> r2{L2, L1, lam_gv<T>(c, 0), lam_gg<T>(c, 0), lam_n,
                              0.25, 0.25 * dt, 1.0, 0.75, 0.0};
  if ((s = adjoint_apply<T>(c, Us[1], B.Gv[1], B.Gg[1], L2, 1, false, nullptr, r2, st))) return s;
  // stage 1: U1 = U + dt R(U):  lam_n += L1 + dt J^T L1
  const hfd::AdjCombine<T> r1{L1, nullptr, nullptr, nullptr, lam_n, 0.0, 0.0, 1.0, 1.0, dt};
  if ((s = adjoint_apply<T>(c, U, B.Gv[0], B.Gg[0], L1, 0, false, nullptr, r1, st))) return s;
  // ghost rows: Dirichlet rows pass lam_{n+1} through, copies carry nothing
  HIPCHK(c, hfd::launch_copy_rows<double>(nd, c->dir_rows, nullptr, nv, A3, lam_n, st));
  HIPCHK(c, hfd::launch_zero_ghost_rows(no + nd, nv, lam_n, st));
  return HFD_OK;
}

hfd_status rk_step_adjoint_impl(hfd_ctx* c, const double* U, const double* U1in,
                                const double* U2in, double dt, const double* lam_np1,
                                double* lam_n, hipStream_t st) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !lam_np1 || !lam_n) return fail(c, HFD_E_INVAL, "null pointer");
  if ((s = ensure_adjoint_t(c))) return s;
  if (mixed(c)) return rk_step_adjoint_t<float>(c, U, U1in, U2in, dt, lam_np1, lam_n, st);
  return rk_step_adjoint_t<double>(c, U, U1in, U2in, dt, lam_np1, lam_n, st);
}

}  // namespace
}  // extern "C++"

hfd_status hfd_rk_step_adjoint(hfd_ctx* c, const double* U, double dt, const double* lam_np1,
                               double* lam_n, void* stream) {
  return rk_step_adjoint_impl(c, U, nullptr, nullptr, dt, lam_np1, lam_n,
                              static_cast<hipStream_t>(stream));
}

hfd_status hfd_rk_step_adjoint_stages(hfd_ctx* c, const double* U, const double* U1,
                                      const double* U2, double dt, const double* lam_np1,
                                      double* lam_n, void* stream) {
  if (!U1 || !U2) return fail(c, HFD_E_INVAL, "null stage state");
  return rk_step_adjoint_impl(c, U, U1, U2, dt, lam_np1, lam_n,
                              static_cast<hipStream_t>(stream));
}

hfd_status hfd_rk_step_stages(hfd_ctx* c, double* U, double dt, double* U1, double* U2,
                              void* stream) {
  hfd_status s = need_device(c);
  if (s) return s;
  if (!U || !U1 || !U2) return fail(c, HFD_E_INVAL, "null state");
  if (mixed(c))
    return rk_step_t<float>(c, c->b32, ecoef32(c), vcoef32(c), true, U, dt, nullptr,
                            static_cast<hipStream_t>(stream), U1, U2);
  return rk_step_t<double>(c, c->b64, ecoef64(c), vcoef64(c), false, U, dt, nullptr,
                           static_cast<hipStream_t>(stream), U1, U2);
}

hfd_status hfd_set_timing(hfd_ctx* c, int32_t on) {
  hfd_status s = need_device(c);
  if (s) return s;
  c->timing = on != 0;
  return HFD_OK;
}

hfd_status hfd_kernel_times(hfd_ctx* c, double* edge_ms, int64_t* n_edge, double* vertex_ms,
                            int64_t* n_vertex) {
  hfd_status s = need_device(c);
  if (s) return s;
  double tot[2] = {0.0, 0.0};
  int64_t cnt[2] = {0, 0};
  for (int k = 0; k < 2; ++k) {
    for (auto& pr : c->ev_pending[k]) {
      HIPCHK(c, hipEventSynchronize(pr.second));
      float ms = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&ms, pr.first, pr.second));
      tot[k] += ms;
      cnt[k] += 1;
      c->ev_pool.push_back(pr.first);
      c->ev_pool.push_back(pr.second);
    }
    c->ev_pending[k].clear();
  }
  if (edge_ms) *edge_ms = tot[0];
  if (n_edge) *n_edge = cnt[0];
  if (vertex_ms) *vertex_ms = tot[1];
  if (n_vertex) *n_vertex = cnt[1];
  return HFD_OK;
}

}  // extern "C"
