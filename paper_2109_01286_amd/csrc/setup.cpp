// Host-side mesh setup.  See setup.h.
//
// Stencil rules (Section 2.1: extend the edge twice from each end along the
// incident edge of smallest deflection; Section 2.3: the divergence stencil
// holds two levels of neighbours and all edges between them), with these
// choices where the paper is silent:
//   - edges oriented from the smaller to the larger input id;
//   - deflection measured by the cosine dot/(|d|*|e|), evaluated in float64
//     in exactly that order (this file is built without FP contraction),
//     largest cosine wins, ties to the smallest input id, vertices already in
//     the stencil excluded, backward extension (i-1, i-2) before forward
//     (i+2, i+3); no candidate is a mesh error;
//   - periodic displacement by the minimum image (d -= P if d > P/2,
//     d += P if d < -P/2);
//   - S(v) = v and its two rings; M(v) = edges with both ends in S(v); an edge
//     is active when some owned vertex uses it.  The slots of S(v) and M(v)
//     are stored in the order of the internal (Hilbert) numbering.
#include "setup.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

namespace hfd {
namespace {

// Stable LSD radix sort of 64-bit keys below 2^bits, 11 bits per pass, with
// an optional payload permuted alongside (empty: none).  Equal keys keep
// their order, so the result equals std::stable_sort by key.
template <class P>
void radix_sort(std::vector<uint64_t>& k, std::vector<P>& pay, int bits) {
  const size_t n = k.size();
  const bool hp = !pay.empty();
  std::vector<uint64_t> k2(n);
  std::vector<P> p2(hp ? n : 0);
  for (int sh = 0; sh < bits; sh += 11) {
    std::vector<size_t> cnt(2049, 0);
    for (size_t i = 0; i < n; ++i) cnt[((k[i] >> sh) & 2047) + 1]++;
    for (int b = 0; b < 2048; ++b) cnt[b + 1] += cnt[b];
    for (size_t i = 0; i < n; ++i) {
      const size_t d = cnt[(k[i] >> sh) & 2047]++;
      k2[d] = k[i];
      if (hp) p2[d] = pay[i];
    }
    k.swap(k2);
    if (hp) pay.swap(p2);
  }
}

int key_bits(uint64_t maxkey) {
  int b = 1;
  while (b < 64 && (maxkey >> b) != 0) ++b;
  return b;
}

inline double minimg(double d, double P) {
  if (P != 0.0) {
    if (d > 0.5 * P) return d - P;
    if (d < -0.5 * P) return d + P;
  }
  return d;
}

struct Geo {
  const double* xy;
  double px, py;
  void disp(int64_t a, int64_t b, double& dx, double& dy) const {
    dx = minimg(xy[2 * b] - xy[2 * a], px);
    dy = minimg(xy[2 * b + 1] - xy[2 * a + 1], py);
  }
};

// Hilbert index of (x, y) on a 2^16 x 2^16 grid.
uint64_t hilbert(uint32_t x, uint32_t y) {
  uint64_t d = 0;
  for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
    uint32_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
    d += uint64_t(s) * uint64_t(s) * ((3 * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - x;
        y = s - 1 - y;
      }
      std::swap(x, y);
    }
  }
  return d;
}

}  // namespace

hfd_status host_setup(const double* xy, int64_t nv, const int32_t* tri,
                      int64_t nt, const int32_t* ghost_src, const hfd_opts& o,
                      HostSetup* out, std::string* err) {
  HostSetup& S = *out;
  S = HostSetup();
  if (!xy || !tri || nv < 3 || nt < 1 || nv > (int64_t(1) << 30)) {
    *err = "invalid mesh sizes or null arrays";
    return HFD_E_INVAL;
  }
  S.nv = nv;
  const Geo geo{xy, o.period[0], o.period[1]};

  // ---- ghost classification ------------------------------------------
  std::vector<int32_t> gs(nv, -1);
  if (ghost_src) std::memcpy(gs.data(), ghost_src, sizeof(int32_t) * nv);
  for (int64_t v = 0; v < nv; ++v) {
    int32_t g = gs[v];
    if (g == -1) continue;
    if (g == -2) continue;
    if (g < 0 || g >= nv || gs[g] != -1) {
      *err = "ghost_src[" + std::to_string(v) + "] is not -1, -2 or an owned vertex";
      return HFD_E_MESH;
    }
  }

  // ---- edges, sorted by (a, b) with a < b ------------------------------
  std::vector<uint64_t> keys;
  keys.reserve(3 * nt);
  for (int64_t t = 0; t < nt; ++t) {
    int64_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv || a == b ||
        b == c || a == c) {
      *err = "triangle " + std::to_string(t) + " has an invalid vertex id";
      return HFD_E_MESH;
    }
    int64_t p[3][2] = {{a, b}, {b, c}, {c, a}};
    for (auto& q : p) {
      uint64_t lo = uint64_t(std::min(q[0], q[1])), hi = uint64_t(std::max(q[0], q[1]));
      keys.push_back(lo * uint64_t(nv) + hi);
    }
  }
  {
    std::vector<int32_t> none;
    radix_sort(keys, none, key_bits(uint64_t(nv) * uint64_t(nv)));
  }
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  const int64_t E = int64_t(keys.size());
  S.ne_mesh = E;
  std::vector<int32_t> ea(E), eb(E);
  for (int64_t e = 0; e < E; ++e) {
    ea[e] = int32_t(keys[e] / uint64_t(nv));
    eb[e] = int32_t(keys[e] % uint64_t(nv));
  }

  // ---- adjacency with edge ids, neighbours sorted ------------------------
  std::vector<int64_t> aptr(nv + 1, 0);
  for (int64_t e = 0; e < E; ++e) {
    aptr[ea[e] + 1]++;
    aptr[eb[e] + 1]++;
  }
  for (int64_t v = 0; v < nv; ++v) aptr[v + 1] += aptr[v];
  std::vector<int32_t> anbr(2 * E), aedge(2 * E);
  {
    std::vector<int64_t> fill(aptr.begin(), aptr.end() - 1);
    // edges are sorted by (a, b): appending in edge order gives, for every
    // vertex, neighbours b > v in increasing order; neighbours a < v also
    // arrive increasing.  Merge the two by a final per-vertex sort.
    for (int64_t e = 0; e < E; ++e) {
      int64_t a = ea[e], b = eb[e];
      anbr[fill[a]] = int32_t(b);
      aedge[fill[a]++] = int32_t(e);
      anbr[fill[b]] = int32_t(a);
      aedge[fill[b]++] = int32_t(e);
    }
    parallel_for(nv, [&](int64_t b0, int64_t b1, unsigned) {
      std::vector<std::pair<int32_t, int32_t>> tmp;
      for (int64_t v = b0; v < b1; ++v) {
        tmp.clear();
        for (int64_t k = aptr[v]; k < aptr[v + 1]; ++k) tmp.emplace_back(anbr[k], aedge[k]);
        std::sort(tmp.begin(), tmp.end());
        for (int64_t k = aptr[v]; k < aptr[v + 1]; ++k) {
          anbr[k] = tmp[k - aptr[v]].first;
          aedge[k] = tmp[k - aptr[v]].second;
        }
      }
    });
  }

  // ---- renumbering: owned, then Dirichlet ghosts, then copying ghosts ----
  std::vector<int32_t> order(nv);
  for (int64_t v = 0; v < nv; ++v) order[v] = int32_t(v);
  auto cls = [&](int64_t v) { return gs[v] == -1 ? 0 : (gs[v] == -2 ? 1 : 2); };
  if (o.order == HFD_ORDER_HILBERT) {
    double x0 = xy[0], x1 = xy[0], y0 = xy[1], y1 = xy[1];
    for (int64_t v = 0; v < nv; ++v) {
      x0 = std::min(x0, xy[2 * v]);
      x1 = std::max(x1, xy[2 * v]);
      y0 = std::min(y0, xy[2 * v + 1]);
      y1 = std::max(y1, xy[2 * v + 1]);
    }
    double sc = 65535.0 / std::max(std::max(x1 - x0, y1 - y0), 1e-300);
    std::vector<uint64_t> hk(nv);
    for (int64_t v = 0; v < nv; ++v) {
      uint32_t ix = uint32_t(std::min(65535.0, std::max(0.0, (xy[2 * v] - x0) * sc)));
      uint32_t iy = uint32_t(std::min(65535.0, std::max(0.0, (xy[2 * v + 1] - y0) * sc)));
      hk[v] = hilbert(ix, iy);
    }
    // by (class, Hilbert key), ties in input order
    for (int64_t v = 0; v < nv; ++v) hk[v] |= uint64_t(cls(v)) << 32;
    radix_sort(hk, order, 34);
  } else if (o.order == HFD_ORDER_RCM) {
    // Reverse Cuthill-McKee over the owned vertices (edges between owned
    // vertices): from a pseudo-peripheral start (repeated breadth-first
    // sweeps to a minimum-degree vertex of the last level), visit the
    // unvisited neighbours by increasing degree (then id), one component
    // after another, and reverse.  Ghost classes keep the input order.
    std::vector<int32_t> deg(nv, 0);
    for (int64_t v = 0; v < nv; ++v)
      if (gs[v] == -1)
        for (int64_t k = aptr[v]; k < aptr[v + 1]; ++k) deg[v] += gs[anbr[k]] == -1;
    std::vector<int32_t> lev(nv, -1), cm;
    cm.reserve(nv);
    auto bfs_levels = [&](int32_t s, std::vector<int32_t>& seen) {  // last level
      std::vector<int32_t> cur{s}, nxt;
      seen.push_back(s);
      lev[s] = 0;
      for (int l = 1;; ++l) {
        nxt.clear();
        for (int32_t u : cur)
          for (int64_t k = aptr[u]; k < aptr[u + 1]; ++k) {
            const int32_t w = anbr[k];
            if (gs[w] == -1 && lev[w] < 0) {
              lev[w] = l;
              seen.push_back(w);
              nxt.push_back(w);
            }
          }
        if (nxt.empty()) return std::make_pair(l - 1, cur);
        std::swap(cur, nxt);
      }
    };
    std::vector<char> done(nv, 0);
    std::vector<int32_t> seen;
    for (int64_t s0 = 0; s0 < nv; ++s0) {
      if (gs[s0] != -1 || done[s0]) continue;
      // pseudo-peripheral vertex of this component
      int32_t start = int32_t(s0);
      int depth = -1;
      for (int it = 0; it < 8; ++it) {
        seen.clear();
        auto [d, last] = bfs_levels(start, seen);
        for (int32_t w : seen) lev[w] = -1;
        int32_t best = last[0];
        for (int32_t w : last)
          if (deg[w] < deg[best] || (deg[w] == deg[best] && w < best)) best = w;
        if (d <= depth) break;
        depth = d;
        start = best;
      }
      // Cuthill-McKee from start
      const size_t c0 = cm.size();
      cm.push_back(start);
      done[start] = 1;
      std::vector<int32_t> nb;
      for (size_t h = c0; h < cm.size(); ++h) {
        const int32_t u = cm[h];
        nb.clear();
        for (int64_t k = aptr[u]; k < aptr[u + 1]; ++k) {
          const int32_t w = anbr[k];
          if (gs[w] == -1 && !done[w]) {
            done[w] = 1;
            nb.push_back(w);
          }
        }
        std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
          return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
        });
        cm.insert(cm.end(), nb.begin(), nb.end());
      }
    }
    std::reverse(cm.begin(), cm.end());
    std::vector<int64_t> rank(nv, 0);
    for (size_t k = 0; k < cm.size(); ++k) rank[cm[k]] = int64_t(k);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      int ca = cls(a), cb = cls(b);
      if (ca != cb) return ca < cb;
      return ca == 0 ? rank[a] < rank[b] : false;
    });
  } else {
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cls(a) < cls(b); });
  }
  S.old_of_new = order;
  S.new_of_old.assign(nv, 0);
  for (int64_t k = 0; k < nv; ++k) S.new_of_old[order[k]] = int32_t(k);
  for (int64_t v = 0; v < nv; ++v) {
    if (gs[v] == -1) S.n_owned++;
    else if (gs[v] == -2) S.n_dir++;
    else S.n_copy++;
  }
  S.gather.resize(nv);
  for (int64_t k = 0; k < nv; ++k) {
    int32_t v = order[k];
    S.gather[k] = gs[v] >= 0 ? S.new_of_old[gs[v]] : int32_t(k);
    if (gs[v] == -2) S.dir_rows.push_back(int32_t(k));
    if (gs[v] >= 0) {
      S.copy_rows.push_back(int32_t(k));
      S.copy_src.push_back(S.new_of_old[gs[v]]);
    }
  }
  const int64_t NO = S.n_owned;

  // ---- two-level vertex stencils of owned vertices (input ids) ----------
  std::vector<std::vector<int32_t>> vn(NO), ve(NO);  // per internal owned vertex
  {
    unsigned ntmax = 16;
    std::vector<std::vector<int32_t>> mark(ntmax, std::vector<int32_t>());
    parallel_for(NO, [&](int64_t b0, int64_t b1, unsigned tid) {
      std::vector<int32_t>& mk = mark[tid];
      mk.assign(nv, -1);
      for (int64_t k = b0; k < b1; ++k) {
        int32_t v = order[k];
        std::vector<int32_t>& s = vn[k];
        s.clear();
        s.push_back(v);
        mk[v] = int32_t(k);
        for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a) {
          int32_t u = anbr[a];
          if (mk[u] != k) { mk[u] = int32_t(k); s.push_back(u); }
        }
        size_t n1 = s.size();
        for (size_t i = 1; i < n1; ++i) {
          int32_t u = s[i];
          for (int64_t a = aptr[u]; a < aptr[u + 1]; ++a) {
            int32_t w = anbr[a];
            if (mk[w] != k) { mk[w] = int32_t(k); s.push_back(w); }
          }
        }
        std::sort(s.begin(), s.end());
        std::vector<int32_t>& m = ve[k];
        m.clear();
        for (int32_t a : s)
          for (int64_t j = aptr[a]; j < aptr[a + 1]; ++j)
            if (anbr[j] > a && mk[anbr[j]] == k) m.push_back(aedge[j]);
        // (a ascending, b ascending within a) == sorted by (a, b) == edge id order
      }
    });
  }

  // ---- active edges in internal order ------------------------------------
  std::vector<uint8_t> active(E, 0);
  for (int64_t k = 0; k < NO; ++k)
    for (int32_t e : ve[k]) active[e] = 1;
  std::vector<uint64_t> ekey;
  std::vector<int32_t> eid;
  for (int64_t e = 0; e < E; ++e)
    if (active[e]) {
      uint64_t p = uint64_t(S.new_of_old[ea[e]]), q = uint64_t(S.new_of_old[eb[e]]);
      if (p > q) std::swap(p, q);
      ekey.push_back(p * uint64_t(nv) + q);
      eid.push_back(int32_t(e));
    }
  // keys are distinct (one per edge)
  if (!eid.empty()) radix_sort(ekey, eid, key_bits(uint64_t(nv) * uint64_t(nv)));
  const int64_t NE = int64_t(eid.size());
  S.ne = NE;
  std::vector<int32_t> e_int(E, -1);
  for (int64_t j = 0; j < NE; ++j) e_int[eid[j]] = int32_t(j);

  // ---- six-node edge stencils ---------------------------------------------
  S.e_end.resize(2 * NE);
  S.e_st.resize(6 * NE);
  std::atomic<int64_t> dead(-1);
  parallel_for(NE, [&](int64_t b0, int64_t b1, unsigned) {
    for (int64_t j = b0; j < b1; ++j) {
      int32_t e = eid[j];
      int32_t a = ea[e], b = eb[e];
      int32_t used[6] = {a, b, -1, -1, -1, -1};
      int nused = 2;
      // next node beyond q on the path p -> q
      auto extend = [&](int32_t p, int32_t q) -> int32_t {
        double dx, dy;
        geo.disp(p, q, dx, dy);
        double dn = std::sqrt(dx * dx + dy * dy);
        int32_t best = -1;
        double bestc = -INFINITY;
        for (int64_t k = aptr[q]; k < aptr[q + 1]; ++k) {
          int32_t c = anbr[k];
          bool u = false;
          for (int t = 0; t < nused; ++t) u |= (used[t] == c);
          if (u) continue;
          double ex, ey;
          geo.disp(q, c, ex, ey);
          double cs = (dx * ex + dy * ey) / (dn * std::sqrt(ex * ex + ey * ey));
          if (cs > bestc) { best = c; bestc = cs; }
        }
        return best;
      };
      int32_t im1 = extend(b, a);
      if (im1 < 0) { dead = j; continue; }
      used[nused++] = im1;
      int32_t im2 = extend(a, im1);
      if (im2 < 0) { dead = j; continue; }
      used[nused++] = im2;
      int32_t ip2 = extend(a, b);
      if (ip2 < 0) { dead = j; continue; }
      used[nused++] = ip2;
      int32_t ip3 = extend(b, ip2);
      if (ip3 < 0) { dead = j; continue; }
      int32_t st[6] = {im2, im1, a, b, ip2, ip3};
      S.e_end[2 * j] = a;
      S.e_end[2 * j + 1] = b;
      for (int t = 0; t < 6; ++t) S.e_st[6 * j + t] = st[t];
    }
  });
  if (dead >= 0) {
    int32_t e = eid[dead];
    *err = "edge (" + std::to_string(ea[e]) + ", " + std::to_string(eb[e]) +
           ") has no six-node stencil (dead end)";
    return HFD_E_MESH;
  }

  // ---- edge frames -------------------------------------------------------
  S.e_stg.resize(6 * NE);
  S.e_pts.resize(12 * NE);
  S.e_h.resize(NE);
  S.e_n.resize(2 * NE);
  parallel_for(NE, [&](int64_t b0, int64_t b1, unsigned) {
    for (int64_t j = b0; j < b1; ++j) {
      const int32_t* st = &S.e_st[6 * j];
      double rx[6], ry[6];
      for (int t = 0; t < 6; ++t) geo.disp(st[2], st[t], rx[t], ry[t]);
      double h = std::hypot(rx[3], ry[3]);
      S.e_h[j] = h;
      S.e_n[2 * j] = rx[3] / h;
      S.e_n[2 * j + 1] = ry[3] / h;
      for (int t = 0; t < 6; ++t) {
        S.e_pts[12 * j + 2 * t] = (rx[t] - 0.5 * rx[3]) / h;
        S.e_pts[12 * j + 2 * t + 1] = (ry[t] - 0.5 * ry[3]) / h;
        S.e_stg[t * NE + j] = S.gather[S.new_of_old[st[t]]];
      }
    }
  });

  // ---- vertex CSR and frames ------------------------------------------------
  S.vptr.assign(NO + 1, 0);
  S.eptr.assign(NO + 1, 0);
  for (int64_t k = 0; k < NO; ++k) {
    S.vptr[k + 1] = S.vptr[k] + int64_t(vn[k].size());
    S.eptr[k + 1] = S.eptr[k] + int64_t(ve[k].size());
    S.max_vs = std::max(S.max_vs, int32_t(vn[k].size()));
    S.max_es = std::max(S.max_es, int32_t(ve[k].size()));
  }
  const int64_t NVS = S.vptr[NO], NES = S.eptr[NO];
  S.v_nodes.resize(NVS);
  S.v_gather.resize(NVS);
  S.v_edges.resize(NES);
  S.v_pts.resize(2 * NVS);
  S.m_pts.resize(2 * NES);
  S.v_h.resize(NO);
  S.v_hmin.resize(NO);
  // Slot order inside a vertex: by gather row (vertex slots) and by internal
  // edge index (edge slots), so that neighbouring lanes gather neighbouring
  // addresses.  The stencil sets are those of the paper's rule; only the
  // order of the terms of the dot products changes.
  parallel_for(NO, [&](int64_t b0, int64_t b1, unsigned) {
    for (int64_t k = b0; k < b1; ++k) {
      std::vector<int32_t>& s = vn[k];
      std::stable_sort(s.begin(), s.end(), [&](int32_t a, int32_t b) {
        return S.gather[S.new_of_old[a]] < S.gather[S.new_of_old[b]] ||
               (S.gather[S.new_of_old[a]] == S.gather[S.new_of_old[b]] &&
                S.new_of_old[a] < S.new_of_old[b]);
      });
      std::vector<int32_t>& m = ve[k];
      std::sort(m.begin(), m.end(), [&](int32_t a, int32_t b) { return e_int[a] < e_int[b]; });
    }
  });
  parallel_for(NO, [&](int64_t b0, int64_t b1, unsigned) {
    for (int64_t k = b0; k < b1; ++k) {
      int32_t v = order[k];
      double hs = 0.0, hm = INFINITY;
      int64_t deg = aptr[v + 1] - aptr[v];
      for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a) {
        double dx, dy;
        geo.disp(v, anbr[a], dx, dy);
        double l = std::hypot(dx, dy);
        hs += l;
        hm = std::min(hm, l);
      }
      double h = hs / double(deg);
      S.v_h[k] = h;
      S.v_hmin[k] = hm;
      int64_t s0 = S.vptr[k];
      for (size_t i = 0; i < vn[k].size(); ++i) {
        int32_t u = vn[k][i];
        double dx, dy;
        geo.disp(v, u, dx, dy);
        S.v_nodes[s0 + i] = u;
        S.v_gather[s0 + i] = S.gather[S.new_of_old[u]];
        S.v_pts[2 * (s0 + i)] = dx / h;
        S.v_pts[2 * (s0 + i) + 1] = dy / h;
      }
      int64_t m0 = S.eptr[k];
      for (size_t i = 0; i < ve[k].size(); ++i) {
        int32_t e = ve[k][i];
        double ax, ay, dx, dy;
        geo.disp(v, ea[e], ax, ay);
        geo.disp(ea[e], eb[e], dx, dy);
        S.v_edges[m0 + i] = e_int[e];
        S.m_pts[2 * (m0 + i)] = (ax + 0.5 * dx) / h;
        S.m_pts[2 * (m0 + i) + 1] = (ay + 0.5 * dy) / h;
      }
    }
  });
  return HFD_OK;
}

}  // namespace hfd
