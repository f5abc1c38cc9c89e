"""The benchmark's path at full size: 864,000 atoms (288,000 waters, 205.0 A box, grid 216^3,
2 A list buffer) along a 0.02 A trajectory, one amoeba_polarize_configuration call per frame in
mixed precision from the previous frame's dipoles and from the learned (delta) start, with the
list kept across the frames.  Every result is compared with an FP64 solve of the same frame to
1e-9 D: rms |mu - mu*| within the 1e-5 D tolerance, E_pol within 1e-6 relative, and the
permanent field on sampled atoms against the oracle."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_2011_01207_amd import amoeba, synth
from parity_util import assert_fields  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def rms_debye(a, b):
    d = (a - b).double()
    return float(4.80320 * torch.sqrt(torch.mean(torch.sum(d * d, dim=1))))


def test_trajectory_steps_match_tightly_converged_fp64():
    s = synth.water864k()
    frames = [torch.tensor(p, device=DEV) for p in synth.trajectory(s, 3, 0.02, seed=77)]
    print(f"[gpu] {s.name}: FP64 references", flush=True)
    fp, t = amoeba.context_for(s, precision="fp64", device=DEV)
    refs = []
    for pos in frames:
        fp.update_blocklist(pos)
        e = fp.perm_field(pos, t["q"], t["dip"], t["quad"])
        mu, ep, it, st = fp.polarize(pos, e, tol_debye=1e-9, max_iter=200)
        assert st == amoeba.AMOEBA_OK
        refs.append((mu, e, ep))
    fp.close()
    idx = np.sort(np.random.default_rng(78).choice(s.n, 128, replace=False))
    s2 = dataclasses.replace(s, pos=frames[2].cpu().numpy())
    e_or = O.perm_field(s2, "spme", idx=idx)
    print(f"[gpu] {s.name}: mixed single-call steps", flush=True)
    mx, _ = amoeba.context_for(s, precision="mixed", device=DEV)
    mx.guess_set_kind("delta")
    mx.guess_set_model(synth.guess_init_model(seed=7))
    try:
        e_out = torch.empty_like(refs[0][1])
        mu0, _, _, _, st, rb = mx.polarize_configuration(frames[0], t["q"], t["dip"], t["quad"], tol_debye=1e-5,
                                                         e_perm_out=e_out)
        assert st == amoeba.AMOEBA_OK and not rb
        prev = (mu0.clone(), e_out.clone())
        for k, mode in ((1, "given"), (2, "learned")):
            if mode == "learned":
                mx.guess_set_reference(*prev)
            mu, _, ep, it, st, rb = mx.polarize_configuration(frames[k], t["q"], t["dip"], t["quad"],
                                                              mu_guess=prev[0] if mode == "given" else None,
                                                              guess_mode=mode, tol_debye=1e-5, e_perm_out=e_out)
            ids = {v: k for k, v in amoeba.GUESS_NAMES.items()}
            assert st == amoeba.AMOEBA_OK and not rb and mx.info()["last_guess"] == ids[mode]
            err = rms_debye(mu, refs[k][0])
            print(f"  frame {k} ({mode} start): {it} it, rms |mu - mu*| {err:.2e} D", flush=True)
            assert err < 1e-5, (k, mode, err)
            assert abs(ep - refs[k][2]) < 1e-6 * abs(refs[k][2])
            prev = (mu.clone(), e_out.clone())
        assert_fields(e_out.cpu().numpy()[idx], e_or, 3e-5, what="E_perm (frame 2) vs oracle")
    finally:
        mx.close()
