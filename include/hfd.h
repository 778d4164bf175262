/*
 * hfd.h -- C ABI of the MI355X (gfx950) implementation of the Hermite
 * finite-difference method for the 2D Euler / Navier-Stokes equations on
 * unstructured triangle meshes (Zhou, Zhen, Qu, Cai, arXiv 2109.01286).
 *
 * The method (Section 2.3, eq. HWENO) evolves the conservative variables
 * w = (rho, rho u, rho v, E) and their gradients w_x, w_y at every vertex.
 * One evaluation of the right-hand side is:
 *   - per edge: a six-node curvilinear stencil (Section 2.1), Hermite
 *     least-squares interpolation of characteristic variables at the edge
 *     midpoint from both sides (Section 2.2, eq. hintp_5), replaced by a
 *     WENO combination of three 3-node interpolations near discontinuities
 *     (eq. 2d_hweno_intp, eq. 3nodes_intp, Algorithm 1), and a Riemann flux
 *     along the edge;
 *   - per vertex: least-squares divergence of the vertex fluxes and edge
 *     fluxes of a two-level stencil (eq. flux_polynomials and the rows
 *     d0, dx, dy that follow it), plus the vertex-only divergence of the
 *     viscous fluxes (Section 2.3, "Computing Viscous Flux");
 *   - the three-stage TVD Runge-Kutta update (end of Section 2.3).
 *
 * Conventions for every entry point below:
 *   - Every call returns an hfd_status; nothing throws across the ABI.  On
 *     failure hfd_last_error(ctx) holds a message.
 *   - State arrays are device memory owned by the caller, float64, layout
 *     U[12][nv] (row q + 4k: q = rho, rho u, rho v, E; k = value, d/dx,
 *     d/dy), in the library's INTERNAL vertex order (see
 *     hfd_permutation).  Mesh arrays passed to hfd_create are host memory
 *     and are copied.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls are stream
 *     ordered and do not synchronise with the host unless stated.
 *   - A context is not thread safe; calls on one context must not overlap.
 */
#ifndef HFD_H
#define HFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hfd_ctx hfd_ctx;

typedef enum {
  HFD_OK = 0,
  HFD_E_INVAL = 1,    /* bad argument (null pointer, size, option value)   */
  HFD_E_MESH = 2,     /* mesh unusable: bad index, dead-end stencil, ...   */
  HFD_E_NOMEM = 3,    /* device or host allocation failed                  */
  HFD_E_DEVICE = 4,   /* HIP runtime error                                 */
  HFD_E_NUMERIC = 5,  /* non-finite value or non-positive rho / p seen     */
  HFD_E_STATE = 6     /* call not valid for this context (e.g. host-only)  */
} hfd_status;

typedef enum { HFD_FP64 = 0, HFD_FP32_MIXED = 1 } hfd_precision;

/* Switch between the 5-node Hermite value and the WENO combination
 * (eq. 2d_hweno_intp): PAPER = Hermite when sw_lo < omega_1 < sw_hi, else
 * WENO; SMOOTH_ONLY / WENO_ONLY force one branch everywhere. */
typedef enum {
  HFD_SWITCH_PAPER = 0,
  HFD_SWITCH_SMOOTH_ONLY = 1,
  HFD_SWITCH_WENO_ONLY = 2
} hfd_switch;

/* Internal numbering of the owned vertices: NONE = input order, HILBERT =
 * along a Hilbert curve of the coordinates (the default), RCM = reverse
 * Cuthill-McKee of the adjacency among owned vertices.  Dirichlet ghosts,
 * then copying ghosts follow in input order.  Results differ only by the
 * order of floating-point sums. */
typedef enum { HFD_ORDER_NONE = 0, HFD_ORDER_HILBERT = 1, HFD_ORDER_RCM = 2 } hfd_order;

/* Riemann flux along the edge (the paper leaves the solver open):
 * RUSANOV = local Lax-Friedrichs; ROE = Roe's flux at the Roe average of the
 * two interface states with Harten's entropy fix on the acoustic waves
 * (|lambda| < d -> (lambda^2 + d^2)/(2 d), d = 0.1 (|u.n| + c)); HLLC = Toro's
 * HLLC flux with the Davis-Einfeldt wave speeds (Roe state). */
typedef enum { HFD_FLUX_RUSANOV = 0, HFD_FLUX_ROE = 1, HFD_FLUX_HLLC = 2 } hfd_flux;

typedef struct hfd_opts {
  double gamma;        /* ratio of specific heats                         */
  double gas_R;        /* gas constant (viscous heat flux only)           */
  double mu;           /* dynamic viscosity; 0 = Euler                    */
  double prandtl;      /* Prandtl number                                  */
  double weno_eps;     /* epsilon of the WENO weights                     */
  double sw_lo, sw_hi; /* open interval of omega_1 for the Hermite branch */
  double w3_cap;       /* > 0: drop singular values of the 3-node systems
                          while a weight exceeds this magnitude; 0 = off  */
  double period[2];    /* period in x and y; 0 = not periodic             */
  double w_ref[4];     /* FP32_MIXED: reference state subtracted from w   */
  int32_t switch_mode; /* hfd_switch                                      */
  int32_t precision;   /* hfd_precision                                   */
  int32_t order;       /* hfd_order: vertex renumbering                   */
  int32_t flux;        /* hfd_flux                                        */
  int32_t stage_off;   /* nonzero: the vertex pass gathers every slot's
                          neighbour data from HBM instead of staging each
                          block's distinct rows and fluxes in LDS, the edge
                          passes every stencil node instead of staging each
                          block's distinct rows, and the edge reverse every
                          entry's lambda rows instead of staging each
                          block's distinct ones (same results bit for bit) */
  int32_t edge_grad;   /* 1: also compute and keep (float64, 96 doubles per
                          edge) the midpoint-derivative rows that
                          hfd_edge_states needs for its grad output; 0: no */
  int32_t deg_inv;     /* degree of the inviscid divergence fit of
                          eq. flux_polynomials: 4 or 5                     */
  int32_t reserved[1];
} hfd_opts;

typedef struct hfd_info {
  int64_t nv;            /* all vertices                                   */
  int64_t n_owned;       /* vertices that are updated (internal 0..n_owned) */
  int64_t n_dirichlet;   /* ghost vertices holding a fixed state            */
  int64_t n_copy_ghost;  /* ghost vertices copying an owned vertex          */
  int64_t n_edges_mesh;  /* edges of the triangulation                      */
  int64_t n_edges;       /* active edges (used by some owned vertex)        */
  int64_t n_vslots;      /* sum over owned v of |S(v)|                      */
  int64_t n_eslots;      /* sum over owned v of |M(v)|                      */
  int32_t max_vslots;    /* max |S(v)|                                      */
  int32_t max_eslots;    /* max |M(v)|                                      */
  int64_t rank_hist[16]; /* edge sides by final Hermite rank                */
  int64_t w3_truncated;  /* 3-node systems with a singular value dropped    */
  /* Algorithmic HBM bytes of one launch at the current precision: every
   * coefficient, index and flux read once, the stage state read once per
   * kernel, outputs written once (second or third Runge-Kutta stage). */
  double bytes_edge_launch;    /* edge pass                              */
  double bytes_vertex_launch;  /* vertex pass with the Runge-Kutta update */
  /* Bytes of the 3-node rows of one edge side, read only when some
   * component of that side takes the 3-node branch (PAPER or SMOOTH switch,
   * or a forced mask); not in bytes_edge_launch.  0 when the rows are
   * always read (WENO everywhere) and counted there. */
  double bytes_edge_w3_side;
  double setup_ms[4];    /* host setup, upload, GPU precompute, total       */
  /* Vertex pass: bytes of a slot's local id when each block of 16 owned
   * vertices stages its distinct state rows and edge fluxes in LDS (1 or 2),
   * 0 when every slot gathers from HBM; the longest such lists. */
  int32_t stage_idx_bytes;
  int32_t stage_max_rows;
  int32_t stage_max_edges;
  int32_t reserved_info;
  /* Bytes the staged vertex pass reads and writes per launch (0 when not
   * staged): bytes_vertex_launch with the local ids, lists and bases in
   * place of the 4-byte slot ids.  bytes_vertex_launch stays the method's
   * figure, with 4-byte ids. */
  double bytes_vertex_staged;
} hfd_info;

/* Default options: gamma 1.4, R 1, mu 0, Pr 0.72, eps 1e-6, (0.01, 0.79),
 * no 3-node cap, not periodic, w_ref 0, PAPER switch, FP64, Hilbert order,
 * Rusanov flux. */
void hfd_default_opts(hfd_opts* o);

const char* hfd_status_string(hfd_status s);
/* Message of the last failure on ctx; with ctx == NULL, of the calling
 * thread's last failed hfd_create. */
const char* hfd_last_error(const hfd_ctx* ctx);

/* Build a context: edges, six-node edge stencils (Section 2.1), two-level
 * vertex stencils (Section 2.3), renumbering, then on the GPU in float64 the
 * Hermite weights (Section 2.2, SVD with the dropping rule), the 3-node
 * weights (eq. 3nodes_intp) and the divergence rows (eq. flux_polynomials)
 * and, if mu > 0, the viscous rows.
 *   xy[nv][2]      vertex coordinates (host)
 *   tri[nt][3]     vertex ids of the triangles (host)
 *   ghost_src[nv]  NULL (no ghosts) or per vertex: -1 owned, -2 ghost with
 *                  a fixed (Dirichlet) state, >= 0 ghost that copies the
 *                  state of that owned vertex (host)
 *   device         HIP device ordinal; -1 builds a host-only context on
 *                  which only the setup queries (info, permutation,
 *                  exports of topology) are valid.
 * Errors: HFD_E_INVAL (sizes, options), HFD_E_MESH (index out of range,
 * ghost source not owned, a stencil with no way forward, a system too
 * large), HFD_E_NOMEM, HFD_E_DEVICE.  On error *out is NULL. */
hfd_status hfd_create(const double* xy, int64_t nv, const int32_t* tri,
                      int64_t nt, const int32_t* ghost_src, const hfd_opts* o,
                      int device, hfd_ctx** out);

hfd_status hfd_destroy(hfd_ctx* ctx);

/* Sizes, statistics and the algorithmic byte model (host, no sync). */
hfd_status hfd_get_info(const hfd_ctx* ctx, hfd_info* out);

/* new_of_old[nv] (host): internal index of every input vertex. */
hfd_status hfd_permutation(const hfd_ctx* ctx, int32_t* new_of_old);

/* Active edges in internal order (host outputs, input vertex ids):
 *   ends[n_edges][2]     (i, i+1): the smaller input id first; n points
 *                        from the first to the second
 *   stencil[n_edges][6]  (i-2, i-1, i, i+1, i+2, i+3) (Section 2.1) */
hfd_status hfd_export_edges(const hfd_ctx* ctx, int32_t* ends, int32_t* stencil);

/* Vertex stencils of the owned vertices in internal order (host outputs):
 *   vptr[n_owned+1], vnodes[n_vslots]  S(v), input vertex ids
 *   eptr[n_owned+1], vedges[n_eslots]  M(v), internal edge indices
 * Slots are in the library's order (by internal index, for coalesced
 * gathers); weight exports and imports use the same slot order. */
hfd_status hfd_export_vertex_stencils(const hfd_ctx* ctx, int64_t* vptr,
                                      int32_t* vnodes, int64_t* eptr,
                                      int32_t* vedges);

/* float64 weights (host outputs, any may be NULL; synchronises):
 *   w5[n_edges][2][15]   Hermite row per side (value, d/dx, d/dy per node,
 *                        side nodes (i-2..i+2) and (i+3..i-1)), physical units
 *   w3[n_edges][2][3][3] 3-node value weights per side and substencil
 *   rank[n_edges][2]     final Hermite rank per side
 *   dv[n_vslots][6]      (d0 f, d0 g, dx f, dx g, dy f, dy g) per stencil node
 *   de[n_eslots][3]      (d0, dx, dy) per stencil edge
 *   dvis[n_vslots][5]    viscous rows (k_x, k_y, k_xx, k_xy, k_yy) per node
 *                        (only when mu > 0) */
hfd_status hfd_export_weights(const hfd_ctx* ctx, double* w5, double* w3,
                              int32_t* rank, double* dv, double* de,
                              double* dvis);

/* Replace the weights (host inputs in the layout of hfd_export_weights; a
 * NULL array keeps the current one).  Refreshes the FP32 copies.
 * Synchronises. */
hfd_status hfd_import_weights(hfd_ctx* ctx, const double* w5, const double* w3,
                              const double* dv, const double* de,
                              const double* dvis);

/* Midpoint-derivative rows (contexts with edge_grad = 1; host arrays,
 * physical units, any may be NULL; synchronise):
 *   w5g[n_edges][2][2][15]   per side and direction (d/dx, d/dy) the
 *                            derivative row of the 5-node operator on
 *                            (value, d/dx, d/dy) of the side's nodes
 *   w3g[n_edges][2][3][2][3] per side, substencil and direction the
 *                            derivative row of the 3-node interpolant
 * Export copies them out; import replaces them (for parity runs with
 * another implementation's rows).  HFD_E_STATE without edge_grad. */
hfd_status hfd_export_grad_weights(const hfd_ctx* ctx, double* w5g, double* w3g);
hfd_status hfd_import_grad_weights(hfd_ctx* ctx, const double* w5g, const double* w3g);

/* Switch the hot path between float64 and the mixed form (float32
 * arithmetic on w - w_ref, float64 Runge-Kutta accumulation).  w_ref[4]
 * (host) is the reference state subtracted before rounding to float32 (NULL
 * keeps the current one).  Allocates the float32 copies of the weights on
 * first use; synchronises. */
hfd_status hfd_set_precision(hfd_ctx* ctx, int32_t precision,
                             const double* w_ref);

/* Riemann flux (hfd_flux) of later residual, step and adjoint calls; the
 * weights do not depend on it.  Errors: HFD_E_INVAL for another value. */
hfd_status hfd_set_flux(hfd_ctx* ctx, int32_t flux);

/* dU = right-hand side of eq. HWENO at state U (device, [12][nv] float64
 * both).  Rows of ghost vertices of dU are set to zero.  Rows of ghost
 * vertices of U are read only for Dirichlet ghosts. */
hfd_status hfd_residual(hfd_ctx* ctx, const double* U, double* dU,
                        void* stream);

/* One three-stage TVD Runge-Kutta step in place on U (device [12][nv]
 * float64).  dt_dev: device pointer to the step size (e.g. written by
 * hfd_stable_dt); rk_step takes it by value.  After the step the rows of
 * copying ghosts hold their source's state. */
hfd_status hfd_rk_step(hfd_ctx* ctx, double* U, double dt, void* stream);
hfd_status hfd_rk_step_dev(hfd_ctx* ctx, double* U, const double* dt_dev,
                           void* stream);

/* nsteps times: hfd_stable_dt(U, cfl) into dt_dev[i], then hfd_rk_step with
 * that step size; dt_dev: device array [nsteps].  The same results bit for
 * bit; between steps the state stays in the passes' gather layout instead of
 * being converted from U again.  U may not be modified by the caller while
 * the call's work runs. */
hfd_status hfd_rk_steps(hfd_ctx* ctx, double* U, int64_t nsteps, double cfl, double* dt_dev,
                        void* stream);

/* *dt_dev = cfl * min over owned v of h_min(v) / (|u_v| + c_v), with h_min
 * the shortest edge at v (device output, no sync). */
hfd_status hfd_stable_dt(hfd_ctx* ctx, const double* U, double cfl,
                         double* dt_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * *dt_dev as hfd_stable_dt, bit for bit, with the per-block partial minima
 * in a scratch array of the library (16384 doubles = 128 KiB per GPU, held
 * until the process ends) instead of the context's buffer.  Calls no
 * allocating routine.  Limit: n_owned <= 4194304 (one partial per 256 owned
 * vertices), else HFD_E_INVAL with a message.  Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (different streams or
 * host threads, any contexts) race and must be serialised by the caller.
 * No sync. */
hfd_status hfd_stable_dt_noalloc(hfd_ctx* ctx, const double* U, double cfl,
                                 double* dt_dev, void* stream);

/* Midpoint states, their derivatives and the flux of every active edge
 * (Section 2.2 / Algorithm 1; device outputs, float64):
 *   wlr[8][n_edges]   rows 0-3 left state (from i-2..i+2), 4-7 right state
 *   grad[16][n_edges] NULL or the derivatives of those states at the edge
 *                     midpoint: row 8 side + 4 d + q = d/dx (d = 0) or d/dy
 *                     (d = 1) of component q of side 0 (left) or 1 (right).
 *                     Per characteristic component, the branch its value
 *                     takes: rows 2 and 3 of the 5-node Hermite operator
 *                     (eq. hintp_5) applied to (c, c_x, c_y), or the
 *                     omega-weighted gradients of the three 3-node
 *                     interpolants (eq. 3nodes_intp); back-projected with R.
 *                     Needs a context created with hfd_opts.edge_grad = 1
 *                     (else HFD_E_STATE).  Not used by the residual.
 *   mask[n_edges]     NULL or bit (4*side + component) set where the WENO
 *                     value was used
 *   h[4][n_edges]     NULL or Riemann flux along the edge direction */
hfd_status hfd_edge_states(hfd_ctx* ctx, const double* U, double* wlr, double* grad,
                           uint8_t* mask, double* h, void* stream);

/* Force the branch of eq. 2d_hweno_intp per edge, side and component:
 * mask_dev[n_edges] (device, bits as in hfd_edge_states) or NULL to return
 * to the configured switch.  The array is referenced, not copied: it must
 * stay valid while forcing is on. */
hfd_status hfd_force_switch_mask(hfd_ctx* ctx, const uint8_t* mask_dev);

/* Copy the state of every copying ghost from its source (device, in place). */
hfd_status hfd_fill_ghosts(hfd_ctx* ctx, double* U, void* stream);

/* Synchronises `stream`; HFD_E_NUMERIC if any residual or step since the
 * last check met a non-finite value or rho <= 0 or p <= 0 at an owned
 * vertex (the flag is then cleared). */
hfd_status hfd_check(hfd_ctx* ctx, void* stream);

/* Adjoint of the residual (Section 2.3, inviscid and, with mu > 0, viscous
 * fluxes): out = (dR/dU)^T lam, all device [12][nv] float64.  Computed in the
 * context's precision: float64, or in HFD_FP32_MIXED float32 arithmetic on
 * the float32 perturbation state of the forward pass, each vertex's sums
 * written in float64.  The
 * branch of eq. 2d_hweno_intp and the WENO weights are differentiated
 * through the branch the forward pass takes, the Rusanov maximum through its
 * larger argument; the Roe and HLLC fluxes by forward-mode dual numbers
 * through the branches they take (entropy fix, wave speeds, HLLC region);
 * the viscous fluxes of a vertex by dual numbers in (w, w_x, w_y).
 * Rows of ghost vertices of out are zero (derivatives with
 * respect to copying ghosts land on their sources; Dirichlet data are
 * constants).  Allocates transposed maps and work buffers on first use. */
hfd_status hfd_adjoint_residual(hfd_ctx* ctx, const double* U, const double* lam,
                                double* out, void* stream);

/* Adjoint of one hfd_rk_step with step size dt (the context's precision for
 * the stage states and adjoint residuals, float64 for the Runge-Kutta
 * combinations of lambda): given the step's
 * input state U_n and lam_np1 = dJ/dU_{n+1}, lam_n = (dU_{n+1}/dU_n)^T
 * lam_np1 (device, [12][nv]).  The two intermediate stages are recomputed.
 * Dirichlet rows of lam_n carry lam_np1 through; rows of copying ghosts are
 * zero.  lam_n may not alias lam_np1. */
hfd_status hfd_rk_step_adjoint(hfd_ctx* ctx, const double* U_n, double dt,
                               const double* lam_np1, double* lam_n, void* stream);

/* One step of hfd_rk_step (the context's precision) that also returns its
 * two intermediate stages (end of Section 2.3):
 * U1 = U + dt R(U), U2 = 3/4 U + 1/4 (U1 + dt R(U1)), device [12][nv]
 * (owned rows; ghost rows unspecified).  For hfd_rk_step_adjoint_stages,
 * which then need not recompute them. */
hfd_status hfd_rk_step_stages(hfd_ctx* ctx, double* U, double dt, double* U1, double* U2,
                              void* stream);

/* hfd_rk_step_adjoint with the step's stages U1, U2 given (as returned by
 * hfd_rk_step_stages from U_n) instead of recomputed.  Same result. */
hfd_status hfd_rk_step_adjoint_stages(hfd_ctx* ctx, const double* U_n, const double* U1,
                                      const double* U2, double dt, const double* lam_np1,
                                      double* lam_n, void* stream);


/* Per-kernel timing, for measurement.  With timing on, every edge pass and
 * every vertex pass launched by hfd_residual / hfd_rk_step* is bracketed by
 * two HIP events recorded on the call's stream.  hfd_kernel_times
 * synchronises on those events and returns, since the previous call, the
 * summed durations in milliseconds and the launch counts of both passes
 * (any output pointer may be NULL), then forgets them. */
hfd_status hfd_set_timing(hfd_ctx* ctx, int32_t on);
hfd_status hfd_kernel_times(hfd_ctx* ctx, double* edge_ms, int64_t* n_edge,
                            double* vertex_ms, int64_t* n_vertex);

#ifdef __cplusplus
}
#endif

#endif /* HFD_H */
