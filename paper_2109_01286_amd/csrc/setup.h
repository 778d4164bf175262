// Host-side mesh setup of the Hermite finite-difference method: edges,
// adjacency, six-node curvilinear edge stencils (Section 2.1), two-level
// vertex stencils (Section 2.3, divergence), renumbering and the local
// frames of every least-squares system.  Plain C++17, deterministic,
// compiled without floating-point contraction so that the stencil choice
// is reproducible bit for bit.
#pragma once

#include <algorithm>
#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/hfd.h"

namespace hfd {

// Allocator that default-initialises (leaves trivial elements unset): the
// large per-slot arrays below are written element by element by parallel
// loops, and a serial zero fill of several GB would dominate the set-up.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <class T>
using HostArray = std::vector<T, NoInitAlloc<T>>;

// f(begin, end, thread) over [0, n) in contiguous chunks on up to 16 threads
// (one call on the calling thread when n is small).
template <class F>
void parallel_for(int64_t n, F&& f) {
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 16) nt = 16;
  if (n < 4096 || nt == 1) {
    f(int64_t(0), n, 0u);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t b = int64_t(t) * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([&f, b, e, t] { f(b, e, t); });
  }
  for (auto& x : th) x.join();
}

struct HostSetup {
  int64_t nv = 0, n_owned = 0, n_dir = 0, n_copy = 0;
  int64_t ne_mesh = 0, ne = 0;
  int32_t max_vs = 0, max_es = 0;

  std::vector<int32_t> new_of_old, old_of_new;  // vertex renumbering
  std::vector<int32_t> gather;        // internal vertex -> row its state is read from
  std::vector<int32_t> dir_rows;      // internal ids of Dirichlet ghosts
  std::vector<int32_t> copy_rows;     // internal ids of copying ghosts
  std::vector<int32_t> copy_src;      // their internal source rows

  // active edges, internal order
  std::vector<int32_t> e_end;         // [ne][2] input ids (i, i+1)
  std::vector<int32_t> e_st;          // [ne][6] input ids (i-2 .. i+3)
  HostArray<int32_t> e_stg;           // [6][ne] gather rows
  HostArray<double> e_pts;            // [ne][6][2] edge frame (midpoint origin, / h_e)
  std::vector<double> e_h;            // [ne] middle-edge length
  std::vector<double> e_n;            // [ne][2] unit direction i -> i+1

  // owned vertices, internal order 0..n_owned-1
  std::vector<int64_t> vptr, eptr;    // [n_owned+1]
  HostArray<int32_t> v_nodes;         // [n_vslots] input ids of S(v)
  HostArray<int32_t> v_gather;        // [n_vslots] gather rows
  HostArray<int32_t> v_edges;         // [n_eslots] internal active-edge index
  HostArray<double> v_pts;            // [n_vslots][2] vertex frame (/ h_v)
  HostArray<double> m_pts;            // [n_eslots][2] edge midpoints, vertex frame
  std::vector<double> v_h;            // [n_owned] mean incident edge length
  std::vector<double> v_hmin;         // [n_owned] shortest incident edge
};

// Returns HFD_OK or an error status with *err set.
hfd_status host_setup(const double* xy, int64_t nv, const int32_t* tri,
                      int64_t nt, const int32_t* ghost_src, const hfd_opts& o,
                      HostSetup* out, std::string* err);

}  // namespace hfd
