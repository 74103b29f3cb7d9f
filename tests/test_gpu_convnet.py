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


@pytest.mark.parametrize("xs,co,K,strides,relu", [
    ((2, 9, 32, 8, 8), 32, 3, (4, 2, 2), True),    # first stage, reduced extents, two channel tiles
    ((3, 8, 9, 5, 6), 8, 3, (2, 1, 1), True),      # ragged
    ((2, 32, 5, 4, 4), 2, 1, (1, 1, 1), False),    # head
    ((1, 3, 7, 7, 7), 20, 3, (1, 1, 1), False),    # channel count not a multiple of 16
])
def test_conv_bf16_matrix_cores(P, xs, co, K, strides, relu):
    """BF16 inference convolution (implicit GEMM on the matrix cores) against
    the oracle's convolution of the BF16-rounded operands: FP32 output within
    1e-5 of the largest magnitude (accumulation order only), BF16 output within
    one BF16 unit of the oracle's rounded value."""
    import torch
    from paper_1504_08340_amd import binding as B
    rng = np.random.default_rng(9)
    x = rng.standard_normal(xs).astype(np.float32)
    w = (rng.standard_normal((co, xs[1], K, K, K)) * 0.3).astype(np.float32)
    b = rng.standard_normal(co).astype(np.float32)
    ref = C.conv3d_forward(C.bf16_round(x), C.bf16_round(w), b.astype(np.float64), strides, relu)
    dev = torch.device("cuda")
    X, Wt, Bt = (torch.tensor(a, device=dev) for a in (x, w, b))
    Xb = torch.empty(X.shape, dtype=torch.bfloat16, device=dev)
    Wb = torch.empty(Wt.shape, dtype=torch.bfloat16, device=dev)
    B.fwi_to_bf16(None, X.numel(), X, Xb)
    B.fwi_to_bf16(None, Wt.numel(), Wt, Wb)
    assert np.array_equal(Xb.float().cpu().numpy(), C.bf16_round(x).astype(np.float32))
    sh = B.conv_shape(*xs, co, K, strides)
    Y32 = torch.empty(ref.shape, dtype=torch.float32, device=dev)
    B.fwi_conv3d_forward_bf16(None, sh, Xb, Wb, Bt, relu, 1, Y32)
    Y16 = torch.empty(ref.shape, dtype=torch.bfloat16, device=dev)
    B.fwi_conv3d_forward_bf16(None, sh, Xb, Wb, Bt, relu, 0, Y16)
    torch.cuda.synchronize()
    _close(Y32.cpu().numpy(), ref)
    got16 = Y16.float().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got16 - C.bf16_round(ref.astype(np.float32))) <= 2.0 ** -7 * np.abs(ref) + 1e-30)


def test_network_bf16_inference_vs_oracle():
    """The shipped network's BF16 forward pass on solver features against
    the oracle's BF16 inference (rounded operands and activations, FP64 sums):
    within 1e-2 relative L2 (hidden activations may round the other way where
    the FP32 and FP64 sums straddle a BF16 boundary); and within 5e-2 of the
    FP32 forward pass, the accuracy BF16 inference gives up."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import os
    from paper_1504_08340_amd import warmstart as WS
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    probe = WS.Probe()
    net = WS.Net.load(os.path.join(root, "paper_1504_08340_amd", "warmstart_weights.npz"), probe.S.device)
    wl = probe.W.with_model(probe.wl, probe.W.layered_profile_vs(probe.wl.prob, 20_003))
    tr = probe.traces(probe.S.tensor(wl.lam_true), probe.S.tensor(wl.mu_true))
    x = torch.empty((1,) + WS.IN_SHAPE, dtype=torch.float32, device=probe.S.device)
    probe.features(tr, net.scale, x[0])
    y16 = net.forward_bf16(x).cpu().numpy().astype(np.float64)
    y32 = net.forward(x)[-1].cpu().numpy().astype(np.float64)
    ref = C.forward_bf16(x.cpu().numpy(), [w.cpu().numpy() for w in net.w], [b.cpu().numpy() for b in net.b],
                         [l[3] for l in WS.LAYERS], [l[4] for l in WS.LAYERS])
    e_ref = np.linalg.norm(y16 - ref) / np.linalg.norm(ref)
    e_32 = np.linalg.norm(y16 - y32) / np.linalg.norm(y32)
    print(f"BF16 inference: vs oracle BF16 {e_ref:.2e}, vs FP32 forward {e_32:.2e}")
    assert e_ref <= 1e-2 and e_32 <= 5e-2
