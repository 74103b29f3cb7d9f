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
    for field, val in (("nsteps", 0), ("npml_side", 0), ("precision", 7), ("ckpt_every", -1)):
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
