"""The C-ABI library loads, exports every symbol its header declares, and
the host-only setup validates its inputs (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2109_01286_amd import hfd, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "hfd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hfd_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = hfd.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hfd.SIGNATURES), "binding and header disagree"


def test_struct_sizes_match_header_layout():
    # hfd_opts: 14 doubles + 8 int32; hfd_info: 8 int64 + 2 int32 + 17 int64 + 7 double
    # + 4 int32 + 1 double
    assert ctypes.sizeof(hfd.Opts) == 14 * 8 + 8 * 4
    assert ctypes.sizeof(hfd.Info) == 8 * 8 + 2 * 4 + 17 * 8 + 7 * 8 + 4 * 4 + 8


def test_default_opts():
    o = hfd.default_opts()
    assert o.gamma == 1.4 and o.weno_eps == 1e-6
    assert o.switch_mode == 0 and o.precision == 0 and o.order == 1
    # the switch interval printed with eq. 2d_hweno_intp, in the library and the oracle
    import os
    from oracle import scheme as osch
    path = os.path.join(os.path.dirname(__file__), "golden", "switch_interval.txt")
    lo, hi = (float(x) for x in next(ln for ln in open(path) if not ln.startswith("#")).split())
    assert (o.sw_lo, o.sw_hi) == (lo, hi)
    assert (osch.Options().sw_lo, osch.Options().sw_hi) == (lo, hi)


def _mesh():
    return inputs.jittered_grid(9, 9, 1.0, 1.0, (False, False), 5, seed=2)


def test_bad_triangle_index_is_a_mesh_error():
    m = _mesh()
    tri = m.tri.copy()
    tri[3, 1] = m.nv + 5
    with pytest.raises(hfd.HfdError) as e:
        hfd.Solver(m.xy, tri, m.ghost_src, m.period, device=-1)
    assert e.value.status == 2 and "triangle 3" in str(e.value)


def test_ghost_source_must_be_owned():
    m = _mesh()
    gs = m.ghost_src.copy()
    g = np.nonzero(gs >= 0)[0]
    gs[g[0]] = g[1]            # a ghost copying another ghost
    with pytest.raises(hfd.HfdError) as e:
        hfd.Solver(m.xy, m.tri, gs, m.period, device=-1)
    assert e.value.status == 2


def test_invalid_options():
    m = _mesh()
    with pytest.raises(hfd.HfdError) as e:
        hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=-1, gamma=0.9)
    assert e.value.status == 1


def test_dead_end_stencil_is_a_mesh_error():
    # a single triangle: no edge can be extended twice
    xy = np.array([[0, 0], [1, 0], [0, 1.0]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    with pytest.raises(hfd.HfdError) as e:
        hfd.Solver(xy, tri, None, (0, 0), device=-1)
    assert e.value.status == 2 and "dead end" in str(e.value)


def test_host_only_context_refuses_device_calls():
    m = _mesh()
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=-1)
    L = hfd.lib()
    assert L.hfd_residual(S._h, None, None, None) == 6
    assert L.hfd_rk_step(S._h, None, 0.1, None) == 6
    assert L.hfd_rk_steps(S._h, None, 3, 0.3, None, None) == 6
    assert L.hfd_adjoint_residual(S._h, None, None, None, None) == 6
    assert S.info["n_owned"] == 81 and S.info["nv"] == 19 * 19


def _stage_lists(ptr, ids, nowned, vpb=16):
    """Sorted distinct ids per block of vpb owned vertices, and the largest
    spread of one vertex's slots over its block's list (brute force)."""
    lists, span = [], 0
    for b in range(0, nowned, vpb):
        lst = np.unique(ids[ptr[b]:ptr[min(nowned, b + vpb)]])
        lists.append(lst)
        for v in range(b, min(nowned, b + vpb)):
            p = np.searchsorted(lst, ids[ptr[v]:ptr[v + 1]])
            span = max(span, int(p.max() - p.min()) + 1)
    return lists, span


def test_vertex_stage_lists_and_byte_model():
    # periodic lattice: no ghosts, so a slot's gather row is its vertex's
    # internal index and the staged lists can be recounted from the export
    m = inputs.jittered_grid(24, 20, 1.0, 1.0, periodic=(True, True), seed=3)
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=-1, precision="fp32")
    S0 = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=-1, precision="fp32",
                    stage_off=1)
    S64 = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=-1)
    i, i0 = S.info, S0.info
    assert i0["stage_idx_bytes"] == 0 and i0["stage_max_rows"] == 0
    assert S64.info["stage_idx_bytes"] == i["stage_idx_bytes"]   # both precisions stage
    vptr, vn, eptr, ve = S.export_vertex_stencils()
    rows, rspan = _stage_lists(vptr, S.new_of_old[vn], S.n_owned)
    edges, espan = _stage_lists(eptr, ve, S.n_owned)
    assert i["stage_max_rows"] == max(len(r) for r in rows)
    assert i["stage_max_edges"] == max(len(e) for e in edges)
    assert i["stage_idx_bytes"] == (1 if max(rspan, espan) <= 256 else 2)
    # bytes of the staged pass: each slot id shrinks from 4 bytes to
    # stage_idx_bytes, and the lists (offsets per block and their entries)
    # and a 4-byte pair of bases per vertex are read once; the method's
    # figure (bytes_vertex_launch) does not depend on the staging
    nb = len(rows)
    lists = 4 * (2 * (nb + 1) + sum(len(r) for r in rows) + sum(len(e) for e in edges)
                 + S.n_owned)
    saved = (4 - i["stage_idx_bytes"]) * (i["n_vslots"] + i["n_eslots"])
    assert i["bytes_vertex_launch"] - i["bytes_vertex_staged"] == pytest.approx(saved - lists, rel=1e-12)
    assert i0["bytes_vertex_staged"] == 0.0
    for k in ("n_vslots", "n_eslots", "bytes_edge_launch", "bytes_vertex_launch", "max_vslots",
              "max_eslots"):
        assert i[k] == i0[k]


def test_binding_refuses_wrong_device_arguments_before_any_launch():
    """The C ABI takes bare pointers, so the binding checks dtype, shape,
    device and layout of every device argument and raises ValueError before
    calling the library (a host-only context: nothing could run anyway)."""
    import torch
    m = _mesh()
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=-1)
    good = torch.zeros(12, S.nv, dtype=torch.float64)
    cases = [
        (lambda: S.residual(good.float()), "dtype"),
        (lambda: S.residual(torch.zeros(4, S.nv, dtype=torch.float64)), "shape"),
        (lambda: S.residual(torch.zeros(12, S.nv + 1, dtype=torch.float64)), "shape"),
        (lambda: S.residual(good), "expected cuda:-1"),
        (lambda: S.residual(good.numpy()), "torch tensor"),
        (lambda: S.rk_step(good, 1e-3), "expected cuda"),
        (lambda: S.rk_steps(good, -1, 0.3), "nsteps"),
        (lambda: S.stable_dt(good, 0.3), "expected cuda"),
        (lambda: S.edge_states(good), "expected cuda"),
        (lambda: S.force_switch_mask(torch.zeros(S.ne, dtype=torch.int32)), "dtype"),
        (lambda: S.force_switch_mask(torch.zeros(S.ne - 1, dtype=torch.uint8)), "shape"),
        (lambda: S.adjoint_residual(good[:, ::2], good), "shape"),
        (lambda: S.rk_step_adjoint(good.float(), 1e-3, good), "dtype"),
        (lambda: S.rk_step_stages(good[:4], 1e-3, good, good), "shape"),
        (lambda: S.rk_step_adjoint_stages(good, good, good, 1e-3, good), "expected cuda"),
        (lambda: S.fill_ghosts(good), "expected cuda"),
    ]
    for call, msg in cases:
        with pytest.raises(ValueError) as e:
            call()
        assert msg in str(e.value), (msg, str(e.value))
    # a transposed view has the right shape but not the layout
    with pytest.raises(ValueError) as e:
        S._state(torch.zeros(S.nv, 12, dtype=torch.float64).t())
    assert "contiguous" in str(e.value) or "expected cuda" in str(e.value)
