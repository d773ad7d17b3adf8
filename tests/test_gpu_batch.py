"""Batched persistent launches (elph_batch_*) against per-context calls.

The persistent kernels run the same tile code as the per-material launches,
so the results must be bitwise equal to elph_scatt_rates on each context
(which the parity tests tie to the oracle); the oracle is also checked
directly on one material.  Graph capture, replay, re-capture at another
temperature and the autotuner are exercised.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import materials as sm

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2109_08547_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _materials():
    out = []
    for name in ("tiny3", "tiny4", "metal6", "plain8"):
        cfg = synth.config(name)
        out.append((cfg, synth.material_for(cfg)))
    mat = sm.make_material(16, 5, 41, sm.rset_cube(-1, 1), sm.rset_cube(0, 1), 2.0, 0.15, 0.6, 0.004)
    out.append((dict(mesh=3, mu=0.0, window=0.9, sigma=0.02, T=300.0), mat))
    return out


def _ctx(cfg, mat, precision):
    return E.elph_create(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"], precision=precision)


def _outputs(ctxs):
    we, wph = [], []
    for c in ctxs:
        sz = E.elph_sizes(c)
        we.append(torch.empty(sz["nstates"], dtype=torch.float64, device=DEV))
        wph.append(torch.empty(sz["nk"] * sz["nbr"], dtype=torch.float64, device=DEV))
    return we, wph


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_contexts(precision):
    mats = _materials()
    T = 300.0
    single = []
    for cfg, mat in mats:
        c = _ctx(cfg, mat, precision)
        E.elph_set_refine(c, 0.0)          # batches run the plain forms (no FP64 refinement)
        sz = E.elph_sizes(c)
        we = torch.empty(sz["nstates"], dtype=torch.float64, device=DEV)
        wph = torch.empty(sz["nk"] * sz["nbr"], dtype=torch.float64, device=DEV)
        E.elph_scatt_rates(c, T, we, wph)
        torch.cuda.synchronize()
        single.append((we.cpu().numpy(), wph.cpu().numpy()))
        c.close()
    ctxs = [_ctx(cfg, mat, precision) for cfg, mat in mats]
    batch = E.elph_batch_create(ctxs)
    # every launch shape the tuner may pick, set explicitly, then the tuner's
    # own pick, with graph capture and replay
    heights = (64, 128) if precision == "fp32" else (128,)
    shapes = [(bpc, so, h) for h in heights for bpc in (1, 2, 4, 8) for so in (0, 1)]
    runs = [("shape", sh, False) for sh in shapes] + [("plain", None, False), ("plain", None, True),
                                                      ("plain", None, True), ("tuned", None, True)]
    for kind, shape, use_graph in runs:
        if kind == "shape":
            E.elph_batch_set_shape(batch, *shape)
        elif kind == "tuned":
            ch = E.elph_batch_tune(batch, T)             # other grids, item orders and tiles, same blocks
            assert ch["tile_rows"] in heights and ch["blocks_per_cu"] in (1, 2, 4, 8)
        we, wph = _outputs(ctxs)
        E.elph_batch_scatt_rates(batch, T, we, wph, use_graph=bool(use_graph))
        torch.cuda.synchronize()
        for m in range(len(mats)):
            assert np.array_equal(we[m].cpu().numpy(), single[m][0]), (kind, shape, use_graph, m)
            assert np.array_equal(wph[m].cpu().numpy(), single[m][1]), (kind, shape, use_graph, m)
    with pytest.raises(E.ElphError) as ei:                # not a candidate shape
        E.elph_batch_set_shape(batch, 3, 1, 128)
    assert ei.value.status == E.elph.ELPH_EINVAL
    batch.close()
    for c in ctxs:
        c.close()


def test_batch_graph_recapture_and_tune_against_oracle():
    mats = _materials()
    ctxs = [_ctx(cfg, mat, "fp64") for cfg, mat in mats]
    batch = E.elph_batch_create(ctxs)
    choice = E.elph_batch_tune(batch, 300.0)
    assert choice["blocks_per_cu"] in (1, 2, 4, 8) and choice["best_ms"] > 0
    cfg, mat = mats[3]                                  # plain8
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    for T in (300.0, 150.0, 300.0):                     # new temperature forces a new graph
        we, wph = _outputs(ctxs)
        E.elph_batch_scatt_rates(batch, T, we, wph, use_graph=True)
        torch.cuda.synchronize()
        Xp, Xm = prob.transition_probs(T)
        ref_we = prob.rates_e(T, Xp, Xm)
        ref_wph = prob.rates_ph(T, Xp).reshape(-1)
        got = we[3].cpu().numpy()
        assert np.abs(got - ref_we).max() <= 1e-10 * np.abs(ref_we).max()
        got = wph[3].cpu().numpy()
        assert np.abs(got - ref_wph).max() <= 1e-10 * np.abs(ref_wph).max()
    # the per-context store left by the batch serves later single calls
    sz = E.elph_sizes(ctxs[3])
    w1 = torch.empty(sz["nstates"], dtype=torch.float64, device=DEV)
    E.elph_scatt_rates(ctxs[3], 300.0, w1, None)
    torch.cuda.synchronize()
    Xp, Xm = prob.transition_probs(300.0)
    ref = prob.rates_e(300.0, Xp, Xm)
    assert np.abs(w1.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
    batch.close()
    for c in ctxs:
        c.close()


def test_batch_rejects_mixed_precision():
    mats = _materials()[:2]
    a = _ctx(*mats[0], "fp64")
    b = _ctx(*mats[1], "fp32")
    with pytest.raises(E.ElphError):
        E.elph_batch_create([a, b])
    a.close()
    b.close()
