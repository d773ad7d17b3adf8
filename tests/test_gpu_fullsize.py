"""Parity at the benchmark's full size (mixed 48^3 workload, launch
configuration of bench.py): outputs the oracle can compute one by one.

W_e of seeded initial states (a row of Eq. 21 needs the vertices of that
state against every final state) and W_ph of seeded phonon modes (Eq. 25
summed over the kept pairs (k, k+q) of each sampled q) are compared with the
plain FP64 path (rel 1e-10) and with the BF16x6, FP32 and FP16x3 forms with
their FP64 refinement (rel 1e-5 on every sampled rate, the strict bar).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2109_08547_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def mixed48():
    cfg = synth.config("mixed48")
    mat = synth.material_for(cfg)
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    T = cfg["T"]
    rng = np.random.default_rng(48)
    rows = np.sort(rng.choice(prob.nstates, 8, replace=False))
    Xp, Xm = prob.transition_probs(T, rows)
    we_rows = prob.rates_e(T, Xp, Xm, rows)
    # q with active modes and kept pairs (k, k+q)
    qs = []
    while len(qs) < 3:
        q = int(rng.integers(1, prob.nq))
        if prob.mode_on[q].any() and q not in qs:
            qs.append(q)
    wph_q = prob.rates_ph_at(T, qs)
    return dict(cfg=cfg, mat=mat, T=T, rows=rows, we=we_rows, qs=qs, wph=wph_q, nstates=prob.nstates)


def _run(c, form):
    cfg = c["cfg"]
    ctx = E.elph_create(c["mat"], cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"], precision=form)
    sz = E.elph_sizes(ctx)
    assert sz["nstates"] == c["nstates"]
    we = torch.empty(sz["nstates"], dtype=torch.float64, device=DEV)
    wph = torch.empty(sz["nk"] * sz["nbr"], dtype=torch.float64, device=DEV)
    E.elph_scatt_rates(ctx, c["T"], we, wph)
    torch.cuda.synchronize()
    nbr = sz["nbr"]
    out = we.cpu().numpy()[c["rows"]], wph.cpu().numpy().reshape(-1, nbr)[c["qs"]]
    ctx.close()
    return out


def _rel(got, ref, floor):
    ref = np.asarray(ref).ravel()
    got = np.asarray(got).ravel()
    big = np.abs(ref) >= floor * np.abs(ref).max()
    return float((np.abs(got[big] - ref[big]) / np.abs(ref[big])).max())


@pytest.mark.parametrize("form,tol,floor", [("fp64", 1e-10, 1e-12), ("bf16x6", 1e-5, 1e-12), ("fp32", 1e-5, 1e-12),
                                             ("fp16x3", 1e-5, 1e-12)])
def test_mixed48_sampled_rates(mixed48, form, tol, floor):
    we, wph = _run(mixed48, form)
    e1 = _rel(we, mixed48["we"], floor)
    e2 = _rel(wph, mixed48["wph"], floor)
    print("\n%s: W_e rows rel err %.2e, W_ph modes rel err %.2e" % (form, e1, e2))
    assert e1 <= tol and e2 <= tol
