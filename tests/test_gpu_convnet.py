"""Warm-start network kernels on the GPU against the FP64 numpy oracle:
convolution forward and its three gradients (strided, with and without ReLU,
3x3x3 and 1x1x1), MSE, Adam, trace features and the coarse-to-node
interpolation.  FP32 kernels: 1e-5 of the largest magnitude."""
import numpy as np
import pytest

import oracle.convnet as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1504_08340_amd as pkg
    return pkg


def _close(got, ref, tol=1e-5):
    got = np.asarray(got, dtype=np.float64)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= tol * max(np.abs(ref).max(), 1e-30)


@pytest.mark.parametrize("xs,co,K,strides,relu", [
    ((2, 9, 32, 8, 8), 8, 3, (4, 2, 2), True),     # first stage, reduced extents
    ((3, 8, 9, 5, 6), 8, 3, (2, 1, 1), True),      # middle stages, ragged
    ((2, 8, 5, 4, 4), 2, 1, (1, 1, 1), False),     # head
    ((1, 3, 7, 7, 7), 4, 3, (1, 1, 1), False),
])
def test_conv_forward_and_backward(P, xs, co, K, strides, relu):
    import torch
    from paper_1504_08340_amd import binding as B
    rng = np.random.default_rng(5)
    x = rng.standard_normal(xs).astype(np.float32)
    w = (rng.standard_normal((co, xs[1], K, K, K)) * 0.3).astype(np.float32)
    b = rng.standard_normal(co).astype(np.float32)
    y_o = C.conv3d_forward(x.astype(np.float64), w.astype(np.float64), b.astype(np.float64), strides, relu)
    dy = rng.standard_normal(y_o.shape).astype(np.float32)
    dx_o, dw_o, db_o = C.conv3d_backward(x.astype(np.float64), w.astype(np.float64), y_o, dy.astype(np.float64),
                                         strides, relu)
    dev = torch.device("cuda")
    X, Wt, Bt, DY = (torch.tensor(a, device=dev) for a in (x, w, b, dy))
    sh = B.conv_shape(*xs, co, K, strides)
    Y = torch.empty(y_o.shape, dtype=torch.float32, device=dev)
    B.fwi_conv3d_forward(None, sh, X, Wt, Bt, relu, Y)
    DX, DW, DB = torch.empty_like(X), torch.empty_like(Wt), torch.empty_like(Bt)
    B.fwi_conv3d_backward(None, sh, X, Wt, Y, DY, relu, DX, DW, DB)
    torch.cuda.synchronize()
    _close(Y.cpu().numpy(), y_o)
    _close(DX.cpu().numpy(), dx_o)
    _close(DW.cpu().numpy(), dw_o)
    _close(DB.cpu().numpy(), db_o)


def test_mse_adam_features_interpolation(P):
    import torch
    from paper_1504_08340_amd import binding as B
    dev = torch.device("cuda")
    rng = np.random.default_rng(6)
    y, t = rng.standard_normal((2, 3000)).astype(np.float32)
    L, G = torch.empty(1, device=dev), torch.empty(3000, device=dev)
    B.fwi_mse(None, 3000, torch.tensor(y, device=dev), torch.tensor(t, device=dev), L, G)
    l_o, g_o = C.mse(y.astype(np.float64), t.astype(np.float64))
    assert abs(float(L[0]) - l_o) <= 1e-5 * l_o
    _close(G.cpu().numpy(), g_o)
    p, g = rng.standard_normal((2, 500)).astype(np.float32)
    m, v = (0.1 * rng.standard_normal((2, 500))).astype(np.float32)
    v = np.abs(v)
    Pt, Mt, Vt = (torch.tensor(a, device=dev) for a in (p, m, v))
    B.fwi_adam(None, 500, Pt, torch.tensor(g, device=dev), Mt, Vt, 1e-2, 0.9, 0.999, 1e-8, 3)
    p_o, m_o, v_o = C.adam_step(*(a.astype(np.float64) for a in (p, g, m, v)), 1e-2, 0.9, 0.999, 1e-8, 3)
    _close(Pt.cpu().numpy(), p_o)
    _close(Mt.cpu().numpy(), m_o)
    _close(Vt.cpu().numpy(), v_o)
    tr = rng.standard_normal((3, 41, 20, 3))
    rec = np.array([7, 0, 19, 3, 11, 5], dtype=np.int32)
    out = torch.empty((3, 12, 6), dtype=torch.float32, device=dev)
    B.fwi_trace_features(None, torch.tensor(tr, device=dev), 3, 40, 20, torch.tensor(rec, device=dev), 6, 12,
                         2, 4, 2, 0.5, out)
    _close(out.cpu().numpy(), C.trace_features(tr, rec, 12, 2, 4, 2, 0.5))
    import workloads as W
    wl = W.tiny(ne_int=(4, 3, 2), npml_side=1, npml_bottom=1, nsteps=3)
    S = P.Solver(wl.prob, wl.src_node, wl.src_dir, wl.rec_node)
    nix, niy, niz = wl.prob.nn_int
    c = (0.1 * rng.standard_normal((3, 4, 5))).astype(np.float32)
    base = rng.uniform(1.0, 2.0, nix * niy * niz)
    o = torch.empty(nix * niy * niz, dtype=torch.float64, device=dev)
    B.fwi_grid_to_nodes(S.plan, None, torch.tensor(c, device=dev), 5, 4, 3, torch.tensor(base, device=dev), o)
    _close(o.cpu().numpy(), C.grid_to_nodes(c.astype(np.float64), nix, niy, niz, base), 1e-6)
    S.close()
