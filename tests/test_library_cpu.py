"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/elph.h declares, and rejects malformed inputs before any
device work."""
import math
import os
import re

import numpy as np
import pytest

import synth

E = pytest.importorskip("paper_2109_08547_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "elph.h")).read()
    return sorted(set(re.findall(r"^\s*(?:elph_status|void|const char\*|int64_t|int32_t)\s+(elph_\w+)\(", src, re.M)))


def test_exports_match_header():
    lib = E.elph.load()
    names = _declared()
    assert set(names) == set(E.elph.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def _mat():
    cfg = synth.config("tiny3")
    return cfg, synth.material_for(cfg)


def _create_status(mat, **kw):
    cfg = synth.config("tiny3")
    args = dict(mesh=cfg["mesh"], mu=cfg["mu"], window=cfg["window"], sigma=cfg["sigma"])
    args.update(kw)
    try:
        ctx = E.elph_create(mat, **args)
    except E.ElphError as e:
        return e.status, e.message
    ctx.close()
    return 0, ""


def test_rejects_non_hermitian_h():
    cfg, mat = _mat()
    mat["h_r"] = mat["h_r"].copy()
    mat["h_r"][1, 0, 1] += 0.3
    st, msg = _create_status(mat)
    assert st == E.elph.ELPH_EINVAL and "Hermitian" in msg


def test_rejects_asr_violation():
    cfg, mat = _mat()
    mat["d_r"] = mat["d_r"].copy()
    mat["d_r"][0] += 0.1 * np.eye(mat["d_r"].shape[1])
    st, msg = _create_status(mat)
    assert st == E.elph.ELPH_EINVAL and "sum rule" in msg


def test_rejects_nan_and_bad_params():
    cfg, mat = _mat()
    bad = dict(mat)
    bad["g_r"] = mat["g_r"].copy()
    bad["g_r"][0, 0, 0, 0, 0] = np.nan
    assert _create_status(bad)[0] == E.elph.ELPH_EINVAL
    assert _create_status(mat, sigma=-1.0)[0] == E.elph.ELPH_EINVAL
    assert _create_status(mat, window=0.0)[0] == E.elph.ELPH_EINVAL
    assert _create_status(mat, mesh=0)[0] == E.elph.ELPH_EINVAL
    assert _create_status(mat, precision=7)[0] == E.elph.ELPH_EINVAL
    assert _create_status(mat, mu=math.nan)[0] == E.elph.ELPH_EINVAL


def test_rejects_unsupported_sizes():
    cfg, mat = _mat()
    big = dict(mat)
    big["natom"] = 6
    assert _create_status(big)[0] == E.elph.ELPH_EINVAL


def test_mlp_create_rejects_bad_shapes_before_device_work():
    prm = np.zeros(10, dtype=np.float32)
    for nin, width, depth in ((0, 64, 1), (8, 100, 1), (8, 64, 0), (8, 64, 9), (2000, 64, 1)):
        with pytest.raises(E.ElphError) as ei:
            E.elph_mlp_create(nin, width, depth, prm)
        assert ei.value.status == E.elph.ELPH_EINVAL


def test_screen_nin_of_null_context_is_zero():
    assert E.elph.load().elph_screen_nin(None) == 0
