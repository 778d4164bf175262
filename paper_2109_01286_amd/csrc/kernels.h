// Launchers of the HIP kernels (internal to libhfd).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hfd.h"

namespace hfd {

// ---- geometric precompute (float64) ----------------------------------------
hipError_t launch_edge_weights(int64_t ne, const double* pts, const double* eh,
                               double w3_cap, double* w5, double* w3,
                               int32_t* rank, int8_t* trunc3, hipStream_t st);
hipError_t launch_div_rows(int64_t nowned, int rpl, const int64_t* vptr,
                           const int64_t* eptr, const double* vpts,
                           const double* mpts, const double* mnrm,
                           const double* vh, double* dv, double* de,
                           int32_t* status, hipStream_t st);
hipError_t launch_visc_rows(int64_t nowned, const int64_t* vptr,
                            const double* vpts, const double* vh, double* dvis,
                            int32_t* status, hipStream_t st);

// ---- hot path ------------------------------------------------------------------
struct GasParams {
  double gamma, gas_R, mu, prandtl;
  double eps, sw_lo, sw_hi;
  double wref[4];   // FP32 form: reference state (zero in the FP64 form)
  int sw;           // hfd_switch
};

// Coefficients of the edge kernel, one precision.
template <class T>
struct EdgeCoef {
  const int32_t* stg;   // [6][ne] gather rows
  const T* n;           // [2][ne]
  const T* w5;          // [2][15][ne]
  const T* w3;          // [2][3][3][ne]
};

template <class T>
struct VertexCoef {
  const int32_t* vptr;     // [n_owned+1] (int32 slot offsets)
  const int32_t* eptr;     // [n_owned+1]
  const int32_t* vg;       // [n_vslots] gather rows
  const int32_t* ve;       // [n_eslots] edge index
  const T* dv;             // [n_vslots][6]
  const T* de;             // [n_eslots][3]
  const T* dvis;           // [n_vslots][5] or null
};

// Gather layout of a stage state: values Gv[nv] and gradients Gg[2 nv]
// (x then y) as 4-vectors, so that one vertex's data is one or two
// contiguous 16/32-byte loads.  In the mixed form it holds w - w_ref.
template <class T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};

// Edge pass: H[ne] (4 components per edge), optional float64 copies
// hsoa[4][ne], states wlr[8][ne] and WENO mask.
template <class T>
hipError_t launch_edge(int64_t ne, const EdgeCoef<T>& c, const GasParams& gp,
                       const V4<T>* Gv, const V4<T>* Gg, const uint8_t* force, V4<T>* H,
                       double* hsoa, double* wlr, uint8_t* mask, hipStream_t st);

// Vertex pass.  mode 0: dU = R (float64 rows [12][nv], owned vertices);
// mode 1: Unew = a*Un + b*(Uk + dt*R) in float64 (dt from dt_dev when
// non-null), plus the gather-layout copy of Unew when Gv_new is non-null.
struct RkArgs {
  const double* Un;
  const double* Uk;
  double* Unew;
  double a, b, dt;
  const double* dt_dev;
};
template <class T>
hipError_t launch_vertex(int64_t nowned, int64_t nv, const VertexCoef<T>& c,
                         const GasParams& gp, const V4<T>* Gv, const V4<T>* Gg,
                         const V4<T>* H, int mode, double* dU, const RkArgs& rk,
                         V4<T>* Gv_new, V4<T>* Gg_new, int32_t* flag, hipStream_t st);

template <class T>
hipError_t launch_to_gather(int64_t nv, const double* U, const GasParams& gp, V4<T>* Gv,
                            V4<T>* Gg, hipStream_t st);
template <class T>
hipError_t launch_copy_gather_rows(int64_t nrows, const int32_t* rows, const V4<T>* fv,
                                   const V4<T>* fg, V4<T>* tv, V4<T>* tg, hipStream_t st);

// Ghost rows and helpers.
template <class T>
hipError_t launch_copy_rows(int64_t nrows, const int32_t* rows, const int32_t* src,
                            int64_t nv, const T* from, T* to, hipStream_t st);
hipError_t launch_zero_ghost_rows(int64_t nowned, int64_t nv, double* dU,
                                  hipStream_t st);
hipError_t launch_stable_dt(int64_t nowned, int64_t nv, const double* U,
                            const double* hmin, double gamma, double cfl,
                            double* partial, int64_t npartial, double* dt,
                            hipStream_t st);
hipError_t launch_cast(int64_t n, const double* a, float* b, hipStream_t st);
hipError_t launch_widen(int64_t n, const float* a, double* b, hipStream_t st);

// ---- adjoint (float64, Euler) ---------------------------------------------------
struct AdjointArgs {
  int64_t ne, nowned, nv;
  const int32_t *etp, *etv, *ets;   // edge m <- (owner vertex, edge slot)
  const double* de;
  const V4<double>* Lv;             // lambda in gather layout
  const V4<double>* Lg;
  V4<double>* lh;                   // [ne] flux adjoint
  EdgeCoef<double> ec;
  GasParams gp;
  const V4<double>* Gv;             // state in gather layout
  const V4<double>* Gg;
  const uint8_t* force;
  double* bnode;                    // [ne][6][12] edge-pass contributions
  const double* U;                  // state [12][nv]
  const int32_t *vtp, *vtv, *vts;   // gather row <- (owner vertex, vertex slot)
  const double* dv;
  const int32_t *ntp, *nte;         // gather row <- (edge, stencil position)
  const int8_t* ntj;
  double* out;                      // [12][nv], owned rows written
};
hipError_t launch_adjoint_residual(const AdjointArgs& a, hipStream_t st);

// out[i] = a x[i] + b y[i] (+ c z[i] if z), i < n
hipError_t launch_axpbypcz(int64_t n, double a, const double* x, double b, const double* y,
                           double c, const double* z, double* out, hipStream_t st);
// lambda of a step's final ghost fill: src rows gather their copies, the
// copies' rows are cleared
hipError_t launch_adj_copy_ghosts(int64_t nsrc, const int32_t* sptr, const int32_t* srows,
                                  const int32_t* gsts, int64_t nv, double* lam,
                                  hipStream_t st);

}  // namespace hfd
