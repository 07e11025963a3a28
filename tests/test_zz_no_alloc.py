"""The allocation-free loss/gradient entry point (mlc_nn_loss_grad_noalloc)
against mlc_nn_loss_grad, through the C ABI: two calls in a row, the second
with fewer rows, each compared with the workspace-backed call on the same
inputs (same kernels and reduction order, so the same values), and both
against the FP64 checker with the bfloat16 roundings of the kernels."""
import ctypes as C

import numpy as np
import pytest

from inputs.nn_init import init_params, random_features
from oracle import learned as Lr

pytestmark = pytest.mark.gpu


def _noalloc(net, X, t):
    from paper_2103_02824_amd import mlc
    L = mlc.lib()
    g = np.zeros(mlc.N_PARAMS, dtype=np.float32)
    loss = C.c_double()
    st = L.mlc_nn_loss_grad_noalloc(net.h, C.c_void_p(X.data_ptr()), C.c_void_p(t.data_ptr()), int(X.shape[0]),
                                    C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float)))
    assert st == 0, (st, L.mlc_nn_last_error(net.h).decode())
    return loss.value, g


def test_noalloc_loss_grad_matches_workspace_call(gpu):
    import torch
    from paper_2103_02824_amd import mlc
    net = mlc.Network()
    th = init_params(3)
    net.set_params(th)
    for k, rows in enumerate((20011, 1007)):
        print(f"case noalloc loss/grad call {k} rows={rows}", flush=True)
        Xn, tn = random_features(40 + k, rows)
        X = torch.from_numpy(Xn).cuda()
        t = torch.from_numpy(tn).cuda()
        l0, g0 = _noalloc(net, X, t)
        l1, g1 = net.loss_grad(X, t)
        print(f"loss {l0} vs {l1}, max |dg| {np.max(np.abs(g0 - g1)):.3e}", flush=True)
        assert abs(l0 - l1) <= 1e-12 * abs(l1)
        assert np.max(np.abs(g0 - g1)) <= 1e-6 * np.max(np.abs(g1))
        lb, gb = Lr.loss_grad(th.astype(np.float64), Xn.astype(np.float64), tn.astype(np.float64), bf=True)
        assert abs(l0 - lb) / lb < 2e-3
        assert np.linalg.norm(g0 - gb) / np.linalg.norm(gb) < 2e-3
    # argument checks: no rows, null outputs
    L = mlc.lib()
    assert L.mlc_nn_loss_grad_noalloc(net.h, C.c_void_p(X.data_ptr()), C.c_void_p(t.data_ptr()), 0, None, None) == -1
    net.close()
