"""GPU check of velo_mlp_grad_noalloc (the gradient for callers that cannot
allocate: partial sums in the library's own device array) against
velo_mlp_grad on the same weights: bit for bit, on two calls in a row, the
second with a smaller input, through the C ABI."""
import ctypes as C
import sys

import numpy as np
import pytest

from gpu_helpers import np_
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _p(t):
    return C.c_void_p(t.data_ptr())


def test_noalloc_grad_matches_context_grad():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = velo.lib()
    rng = np.random.default_rng(404)
    master = rng.normal(0, 0.4, velo.N_PARAM).astype(np.float32)
    norm = np.concatenate([np.zeros(10), np.ones(10)]).astype(np.float32)
    from gpu_helpers import cuts
    v = velo.Velo(gen.plane_z(), cuts("default"))
    v.mlp_set_weights(master, norm)
    d_master = torch.from_numpy(master).cuda()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # the first call spans the largest workgroup count (1024), the second a few
    for n in (70001, 4099):
        say(f"[noalloc] n={n}")
        x = rng.normal(0, 1, (n, 16)).astype(np.float32)
        x[:, 10:] = 0.0
        xb = (x.view(np.uint32) >> 16).astype(np.uint16)  # truncation to BF16 is a valid input too
        feat = torch.from_numpy(xb.view(np.int16)).cuda()
        label = torch.from_numpy((rng.random(n) < 0.3).astype(np.uint8)).cuda()
        g_ref = torch.full((velo.N_PARAM,), float("nan"), device="cuda")
        l_ref = torch.full((1,), float("nan"), device="cuda")
        velo._check(lib.velo_mlp_grad(v.h, n, _p(feat), _p(label), _p(g_ref), _p(l_ref), stream))
        g = torch.full((velo.N_PARAM,), float("nan"), device="cuda")
        loss = torch.full((1,), float("nan"), device="cuda")
        rc = lib.velo_mlp_grad_noalloc(n, _p(d_master), _p(feat), _p(label), _p(g), _p(loss), stream)
        assert rc == 0, lib.velo_last_error()
        torch.cuda.synchronize()
        a, b = np_(g).view(np.int32), np_(g_ref).view(np.int32)
        assert np.isfinite(np_(g)).all()
        assert np.array_equal(a, b), int((a != b).sum())
        assert np.array_equal(np_(loss).view(np.int32), np_(l_ref).view(np.int32))
    # argument errors come back before any device work
    assert lib.velo_mlp_grad_noalloc(0, _p(d_master), _p(feat), _p(label), _p(g), _p(loss), stream) == -1
    assert lib.velo_mlp_grad_noalloc(5, None, _p(feat), _p(label), _p(g), _p(loss), stream) == -1
    v.close()
