"""GPU Kalman fit (velo_kalman_fit) against the oracle.

The device filter performs the oracle's FP32 operations in the same order, so
it must equal the oracle's FP32 filter bit for bit; against the FP64 oracle it
must stay within: positions 1e-5 x max(largest hit radius, 1 mm), slopes 1e-4 x
max(|t|, 1e-3), covariances 1e-3 relative, chi2 1e-3 x max(chi2, 1) (the
FP32 rounding of ~26 filter steps, measured well inside these bounds).
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_helpers import cuts, np_, oracle_run
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def tracks_on_device(b, cut):
    c, t = oracle_run(b, cut)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dev = dict(trk_hit_off=d(t["trk_hit_off"]), trk_hit=d(t["trk_hit"]), trk_planes=d(t["trk_planes"].view(np.int32)),
               clu_x=d(c["clu_x"]), clu_y=d(c["clu_y"]))
    return c, t, dev


def check_close(g, k64, t, c):
    off = np.asarray(t["trk_hit_off"], np.int64)
    hx = c["clu_x"][t["trk_hit"]].astype(np.float64)
    hy = c["clu_y"][t["trk_hit"]].astype(np.float64)
    rmax = np.maximum(np.maximum.reduceat(np.hypot(hx, hy), off[:-1]), 1.0)
    for i in (0, 1):
        assert np.all(np.abs(g[:, i] - k64[:, i]) <= 1e-5 * rmax), f"position {i}"
    for i in (2, 3):
        assert np.all(np.abs(g[:, i] - k64[:, i]) <= 1e-4 * np.maximum(np.abs(k64[:, i]), 1e-3)), f"slope {i}"
    assert np.array_equal(g[:, 4], k64[:, 4].astype(np.float32))
    assert np.allclose(g[:, 5:11], k64[:, 5:11], rtol=1e-3, atol=0)
    assert np.all(np.abs(g[:, 11] - k64[:, 11]) <= 1e-3 * np.maximum(k64[:, 11], 1.0))
    assert np.array_equal(g[:, 12], k64[:, 12])


@pytest.mark.parametrize("name,n,cutname,ms", [("nominal", 120, "ms", 1e-3), ("tiny", None, "default", 0.0),
                                                ("nominal", 60, "ms", 0.0)])
def test_kalman_matches_oracle(velo_mod, name, n, cutname, ms):
    print(f"[kalman] {name} ms={ms}", file=sys.stderr, flush=True)
    w = gen.WORKLOADS[name]
    b = gen.generate(w if n is None else w.with_events(n))
    cut = cuts(cutname)
    c, t, dev = tracks_on_device(b, cut)
    T = len(t["trk_planes"])
    assert T > 0
    v = velo_mod.Velo(b.plane_z, cut)
    g = np_(v.kalman_fit(dev["trk_hit_off"], dev["trk_hit"], dev["trk_planes"], dev["clu_x"], dev["clu_y"], ms,
                         n_tracks=T), T)
    args = (t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], b.plane_z, cut["sigma"], ms)
    k32 = oracle.kalman(*args, fp64=False).astype(np.float32)
    assert np.array_equal(g.view(np.int32), k32.view(np.int32)), "FP32 filter bits"
    check_close(g, oracle.kalman(*args), t, c)
    if ms == 0.0:  # the least-squares line, at the most upstream hit
        f = oracle.fit(t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], b.plane_z,
                       cut["sigma"])
        xl = f[:, 0] + f[:, 3] * (g[:, 4] - f[:, 2])
        assert np.all(np.abs(g[:, 0] - xl) <= 1e-4 * np.maximum(np.abs(xl), 1.0))
        assert np.allclose(g[:, 11], f[:, 5], rtol=1e-3, atol=1e-3)


def test_kalman_on_pipeline_output_with_device_count(velo_mod):
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(50, 4242))
    cut = cuts("ms")
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    out = torch.full((bufs["trk_cap"], 16), -7.0, dtype=torch.float32, device=v.device)
    v.kalman_fit(bufs["trk_hit_off"], bufs["trk_hit"], bufs["trk_planes"], bufs["clu_x"], bufs["clu_y"], 1e-3,
                 max_tracks=bufs["trk_cap"], d_n_tracks=bufs["trk_off"][b.n_events:], out=out)
    torch.cuda.synchronize()
    st = v.read_status(bufs["status"])
    assert st[0] == 0
    T, H = int(st[2]), int(st[3])
    g = np_(out)
    assert np.all(g[T:] == -7.0), "rows beyond the device count untouched"
    n_clu = int(st[1])
    k32 = oracle.kalman(np_(bufs["trk_hit_off"], T + 1), np_(bufs["trk_hit"], H), np_(bufs["trk_planes"], T, np.uint32),
                        np_(bufs["clu_x"], n_clu), np_(bufs["clu_y"], n_clu), b.plane_z, cut["sigma"], 1e-3,
                        fp64=False).astype(np.float32)
    assert np.array_equal(g[:T].view(np.int32), k32.view(np.int32))


def test_kalman_rejects_bad_noise(velo_mod):
    v = velo_mod.Velo(gen.plane_z(), cuts("ms"))
    z = torch.zeros(2, dtype=torch.int32, device="cuda")
    with pytest.raises(velo_mod.VeloError):
        v.kalman_fit(z, z, z, z.float(), z.float(), -1.0, n_tracks=1)
