"""The byte counts behind the bench line's roofline fractions.

Classical RK4 with three registers streams each register value 16 times per
step (stage 1: read the input, which is Xn, write the accumulator and the next
input; stages 2 and 3: read input, Xn and accumulator, write accumulator and
next input; stage 4: read input and accumulator, write Xn), so a forward +
adjoint pass over n_X register values costs 2 x 16 n_X values.  The nodal
launch, averaged over the four stage modes, moves 4 register values per
register entry (3 besides the stage input).  These cases isolate each term.
"""
import types

import pytest

import bench
import workloads as W


def sizes(**kw):
    base = dict(n_nodes=0, n_int_nodes=0, n_pml_nodes=0, n_state=0, n_hist=0)
    base.update(kw)
    return types.SimpleNamespace(**base)


def test_pass_bytes_stream_each_register_value_16_times_per_step():
    # no interior, no nodes: only the registers count (n_X = 2 n_state)
    s = sizes(n_state=1000)
    for es in (4, 8):
        per_dof = bench.pass_bytes_per_dof_step(s, None, 1, es, 0)
        assert per_dof == pytest.approx(2 * 16 * 2 * es, rel=1e-12)   # fwd + adj, 16 passes, n_X = 2 n_state
    # history values join the registers
    assert bench.pass_bytes_per_dof_step(s, None, 1, 4, 500) == pytest.approx(2 * 16 * 4 * (2000 + 500) / 1000, rel=1e-12)


def test_pass_bytes_shared_terms_do_not_scale_with_sources():
    s = sizes(n_state=1000, n_int_nodes=100, n_nodes=300)
    one = bench.pass_bytes_per_dof_step(s, None, 1, 4, 0) * 1000 * 1
    four = bench.pass_bytes_per_dof_step(s, None, 4, 4, 0) * 1000 * 4
    per_src = 2 * 4 * 4 * (4 * 2000 + 3 * 100)
    shared = 2 * 4 * 4 * (2 * 100 + 2 * 300) + 4 * 2 * 2 * 100 * 8
    assert one == pytest.approx(per_src + shared, rel=1e-12)
    assert four == pytest.approx(4 * per_src + shared, rel=1e-12)


def test_nodal_bytes_per_free_node():
    # one more free node (3 more unknowns, one more grid node): per source its
    # 6 register components move 4 times on average over the stage modes
    # (input read + 3), its 3 residual rows are read once, and 1/M once
    prob = W.tiny().prob
    s0 = sizes(n_state=300 + 6 * 40, n_nodes=140, n_int_nodes=50, n_pml_nodes=40)
    s1 = sizes(n_state=303 + 6 * 40, n_nodes=141, n_int_nodes=50, n_pml_nodes=40)
    for es, nsrc in ((4, 1), (4, 3), (8, 2)):
        d = bench.algorithmic_bytes("nodal", s1, prob, nsrc, es) - bench.algorithmic_bytes("nodal", s0, prob, nsrc, es)
        assert d == pytest.approx(es * nsrc * (4 * 6 + 3) + es, rel=1e-12)
