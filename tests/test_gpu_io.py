"""Saved state, error paths and failure recovery of the C ABI (GPU).

* elph_save -> elph_destroy -> elph_create -> elph_load resumes bit for bit:
  the term store, the rates, the coupled iteration at the saving
  temperature and at another one equal those of the uninterrupted context.
* elph_load refuses another material, other parameters, a corrupt or
  truncated file and a missing one (EINVAL); elph_save without a store is
  ESTATE; the context stays usable after each.
* elph_iterate with too small a maxit returns ELPH_ENOCONV with the last
  iterate, and the context then converges normally.
* A device-memory budget forces ELPH_ENOMEM inside elph_scatt_rates and
  inside elph_iterate; the context releases its derived state and, with the
  budget lifted, gives the same results as a fresh one.
"""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2109_08547_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _ctx(name, form="fp64"):
    cfg = synth.config(name)
    mat = synth.material_for(cfg)
    return cfg, E.elph_create(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"], precision=form)


def _bufs(ctx):
    sz = E.elph_sizes(ctx)
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    d = lambda n: torch.empty(int(n), dtype=torch.float64, device=DEV)  # noqa: E731
    return sz, dict(we=d(M), wph=d(nm), I=d(3 * M), J=d(3 * M), F=d(3 * nm), G=d(3 * nm), xp=d(sz["nterms"]))


def _iterate(ctx, b, T, maxit=400, level=None):
    level = E.elph.ELPH_LEVEL_COUPLED if level is None else level
    r = E.elph_iterate(ctx, T, b["I"], b["J"], b["F"], b["G"], level=level, tol=1e-8,
                       maxit=maxit, raise_on_noconv=False)
    torch.cuda.synchronize()
    return r, {k: b[k].cpu().numpy().copy() for k in ("I", "J", "F", "G")}


@pytest.mark.parametrize("form", ["fp64", "fp16x3"])
def test_save_load_resumes_bit_for_bit(tmp_path, form):
    path = str(tmp_path / ("metal6_%s.elph" % form))
    cfg, a = _ctx("metal6", form)
    T = cfg["T"]
    sz, ba = _bufs(a)
    E.elph_scatt_rates(a, T, ba["we"], ba["wph"])
    E.elph_save(a, path)
    assert os.path.getsize(path) > 2 * sz["nterms"] * (8 if form == "fp64" else 4)
    E.elph_transition_probs(a, T, ba["xp"], None, store_B=True)
    ra, outa = _iterate(a, ba, T)
    rb_T2, outa2 = _iterate(a, ba, 200.0)
    we_a, wph_a, xp_a = ba["we"].cpu().numpy().copy(), ba["wph"].cpu().numpy().copy(), ba["xp"].cpu().numpy()
    a.close()
    print("saved %s: %d bytes" % (form, os.path.getsize(path)), flush=True)

    _, b = _ctx("metal6", form)
    _, bb = _bufs(b)
    E.elph_load(b, path)
    E.elph_transition_probs(b, T, bb["xp"], None, store_B=True)
    torch.cuda.synchronize()
    assert np.array_equal(bb["xp"].cpu().numpy(), xp_a)
    rb, outb = _iterate(b, bb, T)
    assert ra["status"] == 0 and rb["status"] == 0 and rb["iters"] == ra["iters"]
    for k in outa:
        assert np.array_equal(outa[k], outb[k]), k
    for t in rb["tensors"]:
        assert np.array_equal(ra["tensors"][t], rb["tensors"][t]), t
    _, outb2 = _iterate(b, bb, 200.0)
    for k in outa2:
        assert np.array_equal(outa2[k], outb2[k]), k
    E.elph_scatt_rates(b, T, bb["we"], bb["wph"])
    torch.cuda.synchronize()
    assert np.array_equal(bb["we"].cpu().numpy(), we_a)
    assert np.array_equal(bb["wph"].cpu().numpy(), wph_a)
    b.close()


def test_load_refuses_other_inputs_and_bad_files(tmp_path):
    path = str(tmp_path / "tiny4.elph")
    cfg, a = _ctx("tiny4")
    _, ba = _bufs(a)
    with pytest.raises(E.ElphError) as ei:                      # nothing to save yet
        E.elph_save(a, path)
    assert ei.value.status == E.elph.ELPH_ESTATE
    E.elph_scatt_rates(a, cfg["T"], ba["we"], ba["wph"])
    torch.cuda.synchronize()
    ref = ba["we"].cpu().numpy().copy()
    E.elph_save(a, path)
    a.close()
    # another material, other parameters, another precision form
    _, other = _ctx("tiny3")
    with pytest.raises(E.ElphError) as ei:
        E.elph_load(other, path)
    assert ei.value.status == E.elph.ELPH_EINVAL
    other.close()
    cfg4 = synth.config("tiny4")
    mat4 = synth.material_for(cfg4)
    for kw in (dict(sigma=cfg4["sigma"] * 2), dict(precision="fp32")):
        args = dict(mesh=cfg4["mesh"], mu=cfg4["mu"], window=cfg4["window"], sigma=cfg4["sigma"])
        args.update(kw)
        c = E.elph_create(mat4, **args)
        with pytest.raises(E.ElphError) as ei:
            E.elph_load(c, path)
        assert ei.value.status == E.elph.ELPH_EINVAL
        c.close()
    mat_g = dict(mat4)
    mat_g["g_r"] = mat4["g_r"] * 1.000001                      # same sizes, other vertex
    c = E.elph_create(mat_g, cfg4["mesh"], cfg4["mu"], cfg4["window"], cfg4["sigma"])
    with pytest.raises(E.ElphError) as ei:
        E.elph_load(c, path)
    assert ei.value.status == E.elph.ELPH_EINVAL and "inputs" in ei.value.message
    c.close()
    # corrupt, truncated and missing files; the context stays usable
    raw = bytearray(open(path, "rb").read())
    bad = str(tmp_path / "bad.elph")
    raw[len(raw) // 2] ^= 0x40
    open(bad, "wb").write(bytes(raw))
    short = str(tmp_path / "short.elph")
    open(short, "wb").write(bytes(raw[: len(raw) // 3]))
    _, c = _ctx("tiny4")
    _, bc = _bufs(c)
    for p in (bad, short, str(tmp_path / "missing.elph")):
        with pytest.raises(E.ElphError) as ei:
            E.elph_load(c, p)
        assert ei.value.status == E.elph.ELPH_EINVAL, p
    E.elph_scatt_rates(c, cfg4["T"], bc["we"], bc["wph"])
    torch.cuda.synchronize()
    assert np.array_equal(bc["we"].cpu().numpy(), ref)
    E.elph_load(c, path)                                      # the good file still loads
    c.close()


def test_iterate_enoconv_returns_the_last_iterate_and_the_context_recovers():
    cfg, a = _ctx("metal6")
    T = cfg["T"]
    _, b = _bufs(a)
    r1, out1 = _iterate(a, b, T, maxit=1, level=E.elph.ELPH_LEVEL_COUPLED)
    assert r1["status"] == E.elph.ELPH_ENOCONV and r1["iters"] == 1
    assert all(np.isfinite(v).all() for v in out1.values())
    assert np.abs(out1["F"]).max() > 0                         # the iterate is there, not zeros
    with pytest.raises(E.ElphError) as ei:                     # raised when asked to
        E.elph_iterate(a, T, b["I"], b["J"], b["F"], b["G"], level=E.elph.ELPH_LEVEL_COUPLED, tol=1e-8, maxit=1)
    assert ei.value.status == E.elph.ELPH_ENOCONV
    r2, out2 = _iterate(a, b, T, level=E.elph.ELPH_LEVEL_COUPLED)
    assert r2["status"] == 0
    a.close()
    _, c = _ctx("metal6")
    _, bc = _bufs(c)
    r3, out3 = _iterate(c, bc, T, level=E.elph.ELPH_LEVEL_COUPLED)
    for k in out2:
        assert np.array_equal(out2[k], out3[k]), k
    c.close()


def test_forced_enomem_releases_and_recovers():
    cfg, fresh = _ctx("metal6", "fp16x3")
    T = cfg["T"]
    _, bf = _bufs(fresh)
    E.elph_scatt_rates(fresh, T, bf["we"], bf["wph"])
    rf, outf = _iterate(fresh, bf, T)
    we_ref = bf["we"].cpu().numpy().copy()
    fresh.close()

    _, a = _ctx("metal6", "fp16x3")
    _, b = _bufs(a)                                           # tables built
    E.elph_set_memory_limit(a, 1 << 40)                       # returns the released blocks to the device
    held = E.elph_memory_held(a)
    E.elph_set_memory_limit(a, held + 1)                      # no new block fits: the store cannot be made
    with pytest.raises(E.ElphError) as ei:
        E.elph_scatt_rates(a, T, b["we"], b["wph"])
    assert ei.value.status == E.elph.ELPH_ENOMEM and "released" in ei.value.message
    assert E.elph_memory_held(a) < held                        # derived tables released too
    E.elph_set_memory_limit(a, 0)
    E.elph_scatt_rates(a, T, b["we"], b["wph"])
    torch.cuda.synchronize()
    assert np.array_equal(b["we"].cpu().numpy(), we_ref)
    # now inside elph_iterate: with the released blocks returned to the
    # device (ELPH_RESET_TRIM) the call must allocate afresh, and cannot
    E.elph_reset(a, E.elph.ELPH_RESET_TRIM)
    E.elph_set_memory_limit(a, E.elph_memory_held(a) + 4096)
    with pytest.raises(E.ElphError) as ei:
        E.elph_iterate(a, T, b["I"], b["J"], b["F"], b["G"], level=E.elph.ELPH_LEVEL_COUPLED, tol=1e-8, maxit=400)
    assert ei.value.status == E.elph.ELPH_ENOMEM
    E.elph_set_memory_limit(a, 0)
    r, out = _iterate(a, b, T)
    assert rf["status"] == 0 and r["status"] == 0 and r["iters"] == rf["iters"]
    for k in out:
        assert np.array_equal(out[k], outf[k]), k
    with pytest.raises(E.ElphError):
        E.elph_set_memory_limit(a, -1)
    a.close()
