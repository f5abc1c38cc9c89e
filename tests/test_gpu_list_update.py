"""The buffered list kept across configurations (amoeba_update_blocklist): no rebuild while
every atom stays within buffer/2 of its position at the last build, a rebuild as soon as one
leaves it, and fields and solves against the oracle at every configuration in between."""
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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_update_keeps_the_list_until_an_atom_leaves_half_the_buffer(prec):
    s0 = dataclasses.replace(synth.water648(), buffer=1.0)
    rng = np.random.default_rng(5)
    print(f"[gpu] list update {prec}", flush=True)
    ctx, t = amoeba.context_for(s0, precision=prec, device=DEV)   # builds at s0
    assert not ctx.update_blocklist(t["pos"])                      # same positions
    tol = {"fp64": 1e-11, "mixed": 2e-5}[prec]
    walk = np.zeros_like(s0.pos)
    for k in range(4):
        walk += rng.normal(0.0, 0.02, s0.pos.shape)
        s = dataclasses.replace(s0, pos=np.mod(s0.pos + walk, s0.box))
        pos = torch.tensor(s.pos, device=DEV)
        assert not ctx.update_blocklist(pos), k                   # max move << 0.5 A
        assert ctx.info()["n_pairs"] == O.count_pairs(s)
        e_ref = O.perm_field(s, "spme")
        e = ctx.perm_field(pos, t["q"], t["dip"], t["quad"])
        assert_fields(e.cpu().numpy(), e_ref, tol, what=f"E_perm frame {k}")
    mu_ref, _, _ = O.pcg(s, e_ref, "spme", tol_debye=1e-10)
    mu, _, _, st = ctx.polarize(pos, e, tol_debye=1e-6)
    assert st == amoeba.AMOEBA_OK and O.rms_debye(mu.cpu().numpy() - mu_ref) < 2e-6
    # one atom 0.6 A from where it was at the build: the list is rebuilt
    far = s.pos.copy()
    far[17] = np.mod(s0.pos[17] + np.array([0.6, 0.0, 0.0]), s0.box)
    s2 = dataclasses.replace(s0, pos=far)
    pos2 = torch.tensor(far, device=DEV)
    with pytest.raises(amoeba.AmoebaError) as ei:                   # the plain calls refuse it
        ctx.perm_field(pos2, t["q"], t["dip"], t["quad"])
    assert ei.value.status == amoeba.AMOEBA_E_LIST
    assert ctx.update_blocklist(pos2)
    assert not ctx.update_blocklist(pos2)
    assert ctx.info()["n_pairs"] == O.count_pairs(s2)
    e2 = ctx.perm_field(pos2, t["q"], t["dip"], t["quad"])
    assert_fields(e2.cpu().numpy(), O.perm_field(s2, "spme"), tol, what="E_perm after the rebuild")
    ctx.close()


def test_update_builds_a_missing_list_and_rejects_bad_positions():
    s = synth.water648()
    ctx = amoeba.Context(s.n, s.box, cutoff=s.cutoff, ewald_alpha=s.ewald_alpha, grid=s.grid, precision="mixed")
    t = torch.tensor(s.pos, device=DEV)
    ctx.set_atoms(*(torch.tensor(a, device=DEV) for a in (s.alpha, s.thole)),
                  torch.tensor(s.sc_ptr, dtype=torch.int32, device=DEV),
                  torch.tensor(s.sc_j, dtype=torch.int32, device=DEV), torch.tensor(s.sc_s, device=DEV))
    assert ctx.update_blocklist(t)
    assert ctx.info()["n_pairs"] == O.count_pairs(s)
    bad = t.clone()
    bad[3, 2] = float("nan")
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.update_blocklist(bad)
    assert ei.value.status == amoeba.AMOEBA_E_NUMERIC
    assert not ctx.update_blocklist(t)      # the list of the last build is still valid
    e = ctx.perm_field(t, *(torch.tensor(a, device=DEV) for a in (s.q, s.dip, s.quad)))
    assert_fields(e.cpu().numpy(), O.perm_field(s, "spme"), 2e-5)
    ctx.close()
