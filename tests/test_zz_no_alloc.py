"""elph_interp_g_noalloc (Eq. 6 at arbitrary pairs without device
allocation) through the C ABI against elph_interp_g on the same inputs (|g|^2
to the FP64 bar 1e-10 of the largest): two calls in a row, the second with
fewer pairs, the first spanning several chunks of the static work array; a
few pairs also against the oracle's |g|^2.  A material whose single pair needs more work space than
the array holds is refused with EINVAL before any device work."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2109_08547_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _pairs(nk, n, seed):
    rng = np.random.default_rng(seed)
    k = rng.integers(0, nk, n).astype(np.int32)
    q = rng.integers(1, nk, n).astype(np.int32)          # q != Gamma (degenerate acoustic modes)
    return k, q


@pytest.mark.parametrize("name,n1,n2", [("plain8", 2000, 37), ("mixed48", 130, 7)])
def test_noalloc_equals_interp_g(name, n1, n2):
    cfg = synth.config(name)
    mat = synth.material_for(cfg)
    print("noalloc: %s, calls of %d then %d pairs" % (name, n1, n2), flush=True)
    ctx = E.elph_create(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    nb, nbr = int(mat["nwann"]), 3 * int(mat["natom"])
    nk = cfg["mesh"] ** 3
    last = None
    for n, seed in ((n1, 1), (n2, 2)):
        k, q = _pairs(nk, n, seed)
        kd, qd = torch.from_numpy(k).to(DEV), torch.from_numpy(q).to(DEV)
        ref = torch.empty((n, nbr, nb, nb, 2), dtype=torch.float64, device=DEV)
        got = torch.full((n, nbr, nb, nb, 2), float("nan"), dtype=torch.float64, device=DEV)
        E.elph_interp_g(ctx, kd, qd, ref)
        E.elph_interp_g_noalloc(ctx, kd, qd, got)
        torch.cuda.synchronize()
        # the same kernels on the same pairs; the chunks differ, and the
        # eigensolver sweeps a wavefront's matrices until all of them have
        # converged, so results agree to rounding: |g|^2 (gauge-free) to the
        # FP64 path's bar
        assert torch.isfinite(got).all(), name
        a = (got ** 2).sum(-1)
        b = (ref ** 2).sum(-1)
        err = ((a - b).abs().max() / b.abs().max()).item()
        print("noalloc: %s, %d pairs: max |d|g|^2| / max|g|^2 = %.2e" % (name, n, err), flush=True)
        assert err <= 1e-10, name
        last = (k, q, got.cpu().numpy())
    ctx.close()
    if name == "plain8":
        k, q, g = last
        kf = oracle.mesh_points(cfg["mesh"])
        g2 = (g ** 2).sum(-1)
        for t in range(5):
            gW = oracle.g_wannier_factorised(mat, kf[k[t]], kf[q[t]][None])[0]
            _, Uk = oracle.electron_bands(mat, kf[k[t]][None])
            _, Ukq = oracle.electron_bands(mat, (kf[k[t]] + kf[q[t]])[None])
            hw, u = oracle.phonon_modes(mat, kf[q[t]][None])
            want = np.abs(oracle.g_bloch(mat, gW, Uk[0], Ukq[0], u[0], hw[0])) ** 2
            assert np.abs(g2[t] - want).max() <= 1e-10 * want.max()


def test_noalloc_refuses_a_pair_larger_than_the_array():
    # 16 bands, 5 atoms, 2197 R_p vectors: one pair needs 2197 * 15 * 256 * 16
    # bytes (135 MB) for its second Wannier stage alone
    nb, na = 16, 5
    nbr = 3 * na
    a = np.arange(-6, 7)
    rp = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    re = np.zeros((1, 3), dtype=np.int32)
    mat = dict(nwann=nb, natom=na, re=re, rp=rp, wre=np.ones(1), wrp=np.ones(len(rp)), lat=5.4 * np.eye(3),
               mass=np.full(na, 28.0855), h_r=np.diag(np.linspace(-1, 1, nb)).astype(complex)[None],
               d_r=np.zeros((len(rp), nbr, nbr)), g_r=np.zeros((1, len(rp), nbr, nb, nb), complex))
    ctx = E.elph_create(mat, 4, 0.0, np.inf, 0.01)
    k = torch.zeros(1, dtype=torch.int32, device=DEV)
    q = torch.ones(1, dtype=torch.int32, device=DEV)
    g = torch.empty((1, nbr, nb, nb, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(E.ElphError) as ei:
        E.elph_interp_g_noalloc(ctx, k, q, g)
    assert ei.value.status == E.elph.ELPH_EINVAL and "work space" in ei.value.message
    # the context stays usable: the allocating entry point still runs
    E.elph_interp_g(ctx, k, q, g)
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    ctx.close()
