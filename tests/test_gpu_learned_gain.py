"""What the trained ghost filters gain over the plain chi2 cut (committed weights).

Both networks were trained on the GPU by the library's own kernels
(paper_2412_05041_amd/train_filter.py).  configs/mlp_default.npz: on
candidates of the single-vertex generator found with the loose windows.  On
independent events of that generator it must keep the efficiency target (>=
plain - 0.5 %) and, there, recover the true tracks the chi2 cut throws away
(those carrying one stray hit) -- a gain of more than a point -- at a ghost
rate still below 0.5 %.  On nominal events (scattering + noise, the ms cut set)
it must keep the efficiency target too.  configs/mlp_nominal.npz: on
candidates of the nominal generator (ghosts weighted 4:1).  On independent
nominal events it must cut the ghost rate below the plain cut's at an
efficiency >= plain - 0.5 %.
"""
import os

import pytest

from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_05041_amd import learned, velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(learned.WEIGHTS):
        pytest.skip("no trained weights")
    master, norm = learned.load_default_weights()
    return learned, velo, master, norm


def test_learned_filter_gain_on_training_like_events(ctx):
    learned, velo, master, norm = ctx
    loose = learned.cuts("loose")
    v = velo.Velo(gen.plane_z(), loose)
    v.mlp_set_weights(master, norm)
    test = gen.generate(gen.WORKLOADS["learned_test"].with_events(2000))
    r = learned.evaluate(v, test, loose, learned.DEFAULT_BAND)
    p, l = r["plain"], r["learned"]
    print(f"plain {p['efficiency']:.4f}/{p['ghost_rate']:.5f}  learned {l['efficiency']:.4f}/{l['ghost_rate']:.5f}")
    assert l["efficiency"] >= p["efficiency"] - 0.005
    assert l["efficiency"] > p["efficiency"] + 0.01
    assert l["ghost_rate"] < 0.005


def test_learned_filter_keeps_nominal_efficiency(ctx):
    learned, velo, master, norm = ctx
    ms = learned.cuts("ms")
    v = velo.Velo(gen.plane_z(), ms)
    v.mlp_set_weights(master, norm)
    nominal = gen.generate(gen.WORKLOADS["nominal"].with_events(200, 9202))
    r = learned.evaluate(v, nominal, ms, learned.DEFAULT_BAND)
    p, l = r["plain"], r["learned"]
    print(f"plain {p['efficiency']:.4f}/{p['ghost_rate']:.5f}  learned {l['efficiency']:.4f}/{l['ghost_rate']:.5f}")
    assert l["efficiency"] >= p["efficiency"] - 0.005
    assert l["ghost_rate"] <= p["ghost_rate"] + 0.005


def test_nominal_filter_cuts_ghosts_at_the_efficiency_target(ctx):
    learned, velo, _, _ = ctx
    if not os.path.exists(learned.NOMINAL_WEIGHTS):
        pytest.skip("no trained nominal weights")
    master, norm = learned.load_default_weights(learned.NOMINAL_WEIGHTS)
    ms = learned.cuts("ms")
    v = velo.Velo(gen.plane_z(), ms)
    v.mlp_set_weights(master, norm)
    nominal = gen.generate(gen.WORKLOADS["nominal"].with_events(400, 9303))
    r = learned.evaluate(v, nominal, ms, learned.DEFAULT_BAND)
    p, l = r["plain"], r["learned"]
    print(f"plain {p['efficiency']:.4f}/{p['ghost_rate']:.5f}  learned {l['efficiency']:.4f}/{l['ghost_rate']:.5f}")
    assert l["efficiency"] >= p["efficiency"] - 0.005
    assert l["ghost_rate"] < p["ghost_rate"]
    assert l["ghost_rate"] < 0.75 * p["ghost_rate"]  # trained: about half
