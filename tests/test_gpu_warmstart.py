"""The learned warm start (the committed network) against the plain start
on a held-out tap trajectory: every step of both runs reaches the 1e-6
residual, and the learned start needs fewer Newton iterations and
assemblies per step.  The network's checkpoint loads without executing
anything and round-trips."""
import os

import numpy as np
import pytest

from gpu_helpers import need_gpu

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CKPT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_24339_amd", "data",
                    "warmstart_mlp.npz")


def test_checkpoint_roundtrip(tmp_path):
    need_gpu()
    from paper_2605_24339_amd import warmstart as W
    net, sc = W.load_checkpoint(CKPT)
    p = str(tmp_path / "ck.npz")
    W.save_checkpoint(p, net, sc)
    net2, sc2 = W.load_checkpoint(p)
    assert torch.equal(net.p, net2.p) and torch.equal(sc.mu, sc2.mu) and torch.equal(sc.ts, sc2.ts)
    x = torch.zeros(100, 16, device="cuda")
    x[:, :9] = torch.randn(100, 9, generator=torch.Generator().manual_seed(0)).cuda()
    assert torch.isfinite(net.predict(sc.x(x))).all()


def test_learned_start_saves_newton_iterations():
    need_gpu()
    from paper_2605_24339_amd import warmstart as W
    net, scaler = W.load_checkpoint(CKPT)
    sc = W.Scene(5045)                 # not among the training trajectories (5000..5019)
    plain = W.run_trajectory(sc, 100, None, keep=False)
    learned = W.run_trajectory(sc, 100, net, keep=False, scaler=scaler, safeguard=True)
    P, L = W.summarize(plain), W.summarize(learned)
    assert P["all_converged"] and L["all_converged"]
    assert L["max_residual"] <= 1e-6 and P["max_residual"] <= 1e-6
    assert L["newton"]["mean"] < P["newton"]["mean"], (L["newton"], P["newton"])
    assert L["assemblies"]["mean"] < P["assemblies"]["mean"]
    # the learned start is closer to the converged solution on average
    assert np.mean([r["start_err"] for r in learned]) < np.mean([r["start_err"] for r in plain])
