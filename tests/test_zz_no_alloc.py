"""ssm_mlp_forward_noalloc, the allocation-free variant of ssm_mlp_forward
(packed weights in the library's static device buffer): through the C ABI,
two calls in a row, the second with fewer rows and other weights, each equal
bitwise to ssm_mlp_forward on the same inputs (the same kernels run on the
same values); an oversized d is refused."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
D = 2
IN = D + 32


def _say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


def test_noalloc_forward_equals_forward():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2105_09688_amd import _lib
    from paper_2105_09688_amd.ssm import mlp_forward, mlp_init
    lib = _lib.load()
    rng = np.random.default_rng(41)
    stream = torch.cuda.current_stream().cuda_stream
    for call, (n, seed) in enumerate(((5000, 1), (777, 2))):
        p = mlp_init(D, seed=seed) + rng.normal(size=mlp_init(D, seed=seed).size).astype(np.float32) * 0.05
        U = np.concatenate([rng.normal(size=(n, D)), rng.uniform(-1, 1, size=(n, 32))], axis=1).astype(np.float32)
        pd = torch.tensor(p, device="cuda")
        Ud = torch.tensor(U, device="cuda")
        ref = mlp_forward(D, pd, Ud).cpu().numpy()
        out = torch.full((n, D), float("nan"), dtype=torch.float32, device="cuda")
        _say(f"call {call}: n={n}")
        st = lib.ssm_mlp_forward_noalloc(D, C.c_void_p(pd.data_ptr()), C.c_void_p(Ud.data_ptr()), n,
                                         C.c_void_p(out.data_ptr()), C.c_void_p(stream))
        assert st == _lib.SSM_OK, lib.ssm_last_error()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), (call, float(np.nanmax(np.abs(got - ref))))
    out = torch.zeros((4, 5), dtype=torch.float32, device="cuda")
    assert lib.ssm_mlp_forward_noalloc(5, C.c_void_p(pd.data_ptr()), C.c_void_p(Ud.data_ptr()), 4,
                                       C.c_void_p(out.data_ptr()), C.c_void_p(stream)) == _lib.SSM_ERR_INVALID
    assert b"d must be in 1..4" in lib.ssm_last_error()
