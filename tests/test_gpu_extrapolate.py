"""GPU forward extrapolation (velo_extrapolate) against the oracle.

Seeded synthetic VELO states and hits (numpy, shared by both sides), an
illustrative magnet; the FP32 device results must agree with the FP64 oracle
within 1e-5 of each quantity's scale (positions: |x0| + |tx| * |z_t - z0| +
window + 1 mm; q/p: the position scale over lever * |kick|).  Also: the device
count of tracks bounds the work, empty input, the pipeline's fit output
chained through the device count, and argument errors.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import cuts, np_
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAG = dict(z_mag=5200.0, z_t=7800.0, kick=1.2, p_min=3.0)  # illustrative, not a detector's


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    p = np.zeros((n, 8), np.float32)
    p[:, 0] = rng.uniform(-40, 40, n)
    p[:, 1] = rng.uniform(-40, 40, n)
    p[:, 2] = rng.uniform(-300, 750, n)
    p[:, 3] = rng.uniform(-0.3, 0.3, n)
    p[:, 4] = rng.uniform(-0.3, 0.3, n)
    qop = rng.uniform(-1 / MAG["p_min"], 1 / MAG["p_min"], n)
    x0, z0, tx = p[:, 0].astype(np.float64), p[:, 2].astype(np.float64), p[:, 3].astype(np.float64)
    xh = (x0 + tx * (MAG["z_mag"] - z0) + (tx + MAG["kick"] * qop) * (MAG["z_t"] - MAG["z_mag"])).astype(np.float32)
    return p, xh


def check(out, ref, p):
    lever = MAG["z_t"] - MAG["z_mag"]
    w = MAG["kick"] / MAG["p_min"] * lever
    scale = (np.abs(p[:, 0]) + np.abs(p[:, 1]) + (np.abs(p[:, 3]) + np.abs(p[:, 4])) * (MAG["z_t"] - p[:, 2])
             + w + 1.0).astype(np.float64)
    o = out.astype(np.float64)
    for col in range(6):
        assert np.all(np.abs(o[:, col] - ref[:, col]) <= 1e-5 * scale), col
    qscale = scale / lever / abs(MAG["kick"])
    assert np.all(np.abs(o[:, 6] - ref[:, 6]) <= 1e-5 * qscale)
    assert np.all(np.abs(o[:, 7] - ref[:, 7]) <= 1e-5 * (np.abs(ref[:, 7]) + qscale * abs(MAG["kick"])))


def test_matches_oracle(velo_mod):
    n = 100_003
    p, xh = inputs(n, 5)
    v = velo_mod.Velo(gen.plane_z(), cuts("ms"))
    d = lambda a: torch.from_numpy(a).cuda()
    out = np_(v.extrapolate(d(p), MAG, x_hit=d(xh)), n)
    check(out, oracle.extrapolate(p, xh, **MAG), p)
    out0 = np_(v.extrapolate(d(p), MAG), n)
    ref0 = oracle.extrapolate(p, None, **MAG)
    check(out0, ref0, p)
    assert np.all(out0[:, 6] == 0)


def test_device_count_and_empty(velo_mod):
    p, xh = inputs(1000, 6)
    v = velo_mod.Velo(gen.plane_z(), cuts("ms"))
    d = lambda a: torch.from_numpy(a).cuda()
    out = torch.full((1000, 8), -7.0, dtype=torch.float32, device="cuda")
    cnt = torch.tensor([600], dtype=torch.int32, device="cuda")
    v.extrapolate(d(p), MAG, x_hit=d(xh), max_tracks=1000, d_n_tracks=cnt, out=out)
    o = np_(out)
    check(o[:600], oracle.extrapolate(p[:600], xh[:600], **MAG), p[:600])
    assert np.all(o[600:] == -7.0)
    v.extrapolate(d(p), MAG, max_tracks=0, out=out)  # nothing to do
    torch.cuda.synchronize()


def test_chained_on_the_pipeline_fit(velo_mod):
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(50, 31))
    v = velo_mod.Velo(b.plane_z, cuts("ms"))
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    out = v.extrapolate(bufs["par"], MAG, max_tracks=bufs["trk_cap"], d_n_tracks=bufs["trk_off"][b.n_events:])
    T = int(bufs["trk_off"][-1].item())
    par = np_(bufs["par"], T)
    check(np_(out, T), oracle.extrapolate(par, None, **MAG), par)


@pytest.mark.parametrize("bad", [dict(z_t=5000.0), dict(kick=0.0), dict(p_min=0.0), dict(p_min=float("nan"))])
def test_argument_errors(velo_mod, bad):
    p, _ = inputs(10, 7)
    v = velo_mod.Velo(gen.plane_z(), cuts("ms"))
    with pytest.raises(velo_mod.VeloError):
        v.extrapolate(torch.from_numpy(p).cuda(), dict(MAG, **bad))
