"""The C-ABI library loads and exports every symbol include/pmlfwi.h declares
(no GPU compute here; fwi_query is a host-only function)."""
import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmlfwi.h")
LIB = os.path.join(ROOT, "paper_1504_08340_amd", "libpmlfwi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fwi_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpmlfwi.so not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fwi_query", "fwi_plan_create", "fwi_plan_destroy", "fwi_forward", "fwi_misfit",
              "fwi_adjoint_gradient", "fwi_apply_operator", "fwi_status_string", "fwi_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_1504_08340_amd import binding
    assert sorted(binding.EXPORTS) == declared_functions()


@pytest.mark.parametrize("name,make,nsrc", [("cfg1", W.config1, 1), ("tiny", W.tiny, 1)])
def test_query_sizes_match_oracle_mesh(name, make, nsrc):
    from oracle.mesh import Mesh
    from paper_1504_08340_amd import binding
    wl = make()
    s = binding.fwi_query(binding.make_problem(wl.prob, nsrc, wl.nrec))
    m = Mesh(wl.prob)
    assert s.n_state == m.n_state and s.n_hist == m.n_hist
    assert s.n_nodes == m.n_nodes and s.n_int_nodes == m.n_int_nodes
    assert s.n_pml_nodes == int(m.in_pml.sum())
    assert s.trace_len == nsrc * (wl.prob.nsteps + 1) * wl.nrec * 3


def test_query_rejects_bad_problems():
    from paper_1504_08340_amd import binding
    wl = W.tiny()
    for field, val in (("nsteps", 0), ("npml_side", 0), ("precision", 7), ("ckpt_every", -2)):
        p = binding.make_problem(wl.prob, 1, wl.nrec)
        setattr(p, field, val)
        with pytest.raises(binding.FwiError):
            binding.fwi_query(p)


def test_checkpoint_spacing_shrinks_the_workspace():
    """40x40x20 m mesh, 4 sources, 2000 steps, FP64: keeping a full state every k
    steps (and one segment of stage displacements) instead of every stage."""
    from paper_1504_08340_amd import binding
    wl = W.config2(nsteps=2000)

    def ws(k):
        return binding.fwi_query(binding.make_problem(wl.prob, 4, wl.nrec, 0, k)).workspace_bytes

    full = ws(0)
    sizes = {k: ws(k) for k in (10, 50, 200)}
    print({k: f"{v / 2**30:.1f} GiB" for k, v in sizes.items()}, f"k=0: {full / 2**30:.1f} GiB")
    assert all(v * 3 < full for v in sizes.values())
    assert sizes[50] < sizes[10] and sizes[50] < sizes[200]


@pytest.mark.parametrize("name, make", [("tiny_ragged", lambda: W.tiny(ne_int=(3, 2, 3), npml_side=2, npml_bottom=1)),
                                        ("cfg2", lambda: W.config2(nsteps=10))])
def test_query_reports_a_tiling_that_covers_the_bricks(name, make):
    """The element tiles reported by fwi_query partition the bricks: each tile
    holds at most tile[0] x tile[1] x tile[2] bricks, interior and PML tiles
    together cover every brick, and a workgroup holds the tile's node box."""
    from paper_1504_08340_amd import binding
    wl = make()
    q = binding.fwi_query(binding.make_problem(wl.prob, 1, wl.nrec, 1, 0))
    tx, ty, tz = q.tile
    ex, ey, ez = wl.prob.ne_int
    ps, pb = wl.prob.npml_side, wl.prob.npml_bottom
    assert q.element_threads >= (2 * tx + 1) * (2 * ty + 1) * (2 * tz + 1)
    assert q.tiles_interior == -(-ex // tx) * -(-ey // ty) * -(-ez // tz)
    bricks = (ex + 2 * ps) * (ey + 2 * ps) * (ez + pb)
    per_axis = [-(-ps // tx) * 2 + -(-ex // tx), -(-ps // ty) * 2 + -(-ey // ty), -(-pb // tz) + -(-ez // tz)]
    assert q.tiles_interior + q.tiles_pml == per_axis[0] * per_axis[1] * per_axis[2]
    assert (q.tiles_interior + q.tiles_pml) * tx * ty * tz >= bricks
