"""The allocation-free gradient entry point (nbgs_mlp_loss_grad_static) through the C ABI: two calls in a row, the
second with fewer samples (the fixed scratch keeps the first call's partials, which must not leak into the second),
each against nbgs_mlp_loss_grad on the same network and inputs, bit for bit; sizes past its limit are refused."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def test_static_scratch_gradient_equals_the_workspace_one():
    import torch

    nb = _nb()
    rng = np.random.default_rng(17)
    mlp = nb.GpuMlp(seed=11)
    L = nb.lib()
    npar = nb.nbgs_mlp_param_count()
    for n in (4096, 700):  # the largest size, then a smaller one over the same scratch
        x = torch.tensor(rng.normal(size=(n, 12)).astype(np.float32), device="cuda")
        t = torch.tensor(rng.normal(size=(n, 3)).astype(np.float32), device="cuda")
        g_ref = torch.empty(npar, dtype=torch.float32, device="cuda")
        g_st = torch.full((npar,), float("nan"), dtype=torch.float32, device="cuda")
        l_ref, l_st = C.c_double(), C.c_double()
        assert L.nbgs_mlp_loss_grad(C.c_void_p(mlp.handle), C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                    n, C.c_void_p(g_ref.data_ptr()), C.byref(l_ref)) == 0
        assert L.nbgs_mlp_loss_grad_static(C.c_void_p(mlp.handle), C.c_void_p(x.data_ptr()),
                                           C.c_void_p(t.data_ptr()), n, C.c_void_p(g_st.data_ptr()),
                                           C.byref(l_st)) == 0, nb.nbgs_last_error()
        torch.cuda.synchronize()
        assert np.array_equal(g_st.cpu().numpy(), g_ref.cpu().numpy()), n
        assert l_st.value == l_ref.value and l_st.value > 0.0
    # refused past its limit, and without an output
    x = torch.zeros((4097, 12), dtype=torch.float32, device="cuda")
    t = torch.zeros((4097, 3), dtype=torch.float32, device="cuda")
    g = torch.empty(npar, dtype=torch.float32, device="cuda")
    assert L.nbgs_mlp_loss_grad_static(C.c_void_p(mlp.handle), C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                       4097, C.c_void_p(g.data_ptr()), None) == 1
    assert "4096" in nb.nbgs_last_error()
    assert L.nbgs_mlp_loss_grad_static(C.c_void_p(mlp.handle), C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                       10, None, None) == 1
    mlp.close()
