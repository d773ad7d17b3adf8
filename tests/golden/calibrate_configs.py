"""Write synth/configs.json: the calibrated scales of every named workload.

Uses only the oracle (band energies, phonon energies) and the input
generator.  For each workload:

* c_D scales the force constants so that the largest hbar*omega on the run's
  q mesh is 60 meV;
* delta (the on-site offset of the lower/upper half of the bands) is bisected
  so that the gap CBM - VBM on the run's k mesh is 1.0 eV, with
  VBM = max of band nb/2 - 1 and CBM = min of band nb/2 (0-based);
* where a kept fraction is targeted, s_H is bisected (log scale) so that the
  fraction of k with any band within +-window of mu is the target;
* mu = midgap + 0.1 eV or CBM - 0.1 eV as the workload states.

Run:  python tests/golden/calibrate_configs.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import materials as sm  # noqa: E402

OUT = os.path.join(ROOT, "synth", "configs.json")
HW_MAX = 0.060
GAP = 1.0


def _bands(h_raw_k, onsite, s_H, delta):
    h = s_H * h_raw_k + np.diag(onsite * delta)[None]
    return np.linalg.eigvalsh(h)


def _raw_hk(cfg, kfrac):
    mat = sm.material_for(cfg, s_H=1.0, delta=0.0, c_D=1.0, with_g=False)
    out = np.empty((kfrac.shape[0], cfg["nb"], cfg["nb"]), dtype=np.complex128)
    for s in range(0, kfrac.shape[0], 32768):
        out[s:s + 32768] = oracle.bloch_hamiltonian(mat, kfrac[s:s + 32768])
    return mat, out


def _gap_delta(hk, onsite, s_H, nb):
    """Bracketed Illinois (regula falsi) iteration on gap(delta) = GAP; the
    gap grows with delta."""
    def gap(delta):
        e = _bands(hk, onsite, s_H, delta)
        return e[:, nb // 2].min() - e[:, nb // 2 - 1].max() - GAP
    lo, hi = 0.0, 1.0
    flo, fhi = gap(lo), gap(hi)
    while fhi < 0:
        lo, flo = hi, fhi
        hi *= 2.0
        fhi = gap(hi)
    side = 0
    x = hi
    for _ in range(100):
        x = (lo * fhi - hi * flo) / (fhi - flo)
        fx = gap(x)
        if abs(fx) < 1e-11 or hi - lo < 1e-13:
            return x
        if fx > 0:
            hi, fhi = x, fx
            if side == 1:
                flo *= 0.5
            side = 1
        else:
            lo, flo = x, fx
            if side == -1:
                fhi *= 0.5
            side = -1
    raise RuntimeError("gap calibration did not converge")


def calibrate(name, sub=1):
    """``sub`` > 1 bisects s_H on every sub-th mesh point per axis (the final
    gap, mu and kept fraction are taken on the full mesh)."""
    t0 = time.time()
    cfg = synth.config(name, calibrated=False)
    nb = cfg["nb"]
    kfrac = oracle.mesh_points(cfg["mesh"])
    mat, hk = _raw_hk(cfg, kfrac)
    onsite = np.array([-1.0 if b < nb // 2 else 1.0 for b in range(nb)])
    n = cfg["mesh"]
    ijk = np.rint(kfrac * n).astype(int)
    coarse = np.all(ijk % sub == 0, axis=1)
    hk_full = hk

    # force-constant scale from the raw Gram matrices
    lam_max = 0.0
    for s in range(0, kfrac.shape[0], 32768):
        d = oracle.dynamical_matrix(mat, kfrac[s:s + 32768])
        lam_max = max(lam_max, float(np.linalg.eigvalsh(d).max()))
    c_D = HW_MAX ** 2 / (oracle.C_PHONON * lam_max)

    def solve(s_H, hk=hk_full):
        if "delta_fixed" in cfg:
            delta = float(cfg["delta_fixed"])
        else:
            delta = _gap_delta(hk, onsite, s_H, nb)
        e = _bands(hk, onsite, s_H, delta)
        vbm = e[:, max(nb // 2 - 1, 0)].max()
        cbm = e[:, nb // 2].min()
        if cfg["mu_rule"] == "median":
            mu = float(np.median(e))
        elif cfg["mu_rule"] == "midgap+0.1":
            mu = 0.5 * (vbm + cbm) + 0.1
        elif cfg["mu_rule"] == "cbm-0.1":
            mu = cbm - 0.1
        else:
            raise ValueError(cfg["mu_rule"])
        kept = float((np.abs(e - mu) <= cfg["window"]).any(1).mean())
        return delta, mu, kept, vbm, cbm

    if "kept_target" in cfg:
        target = cfg["kept_target"]
        lo, hi = np.log(0.005), np.log(2.0)
        # kept fraction falls as s_H grows (more dispersive bands)
        hk_c = hk_full[coarse]
        for _ in range(40):
            mid = 0.5 * (lo + hi)
            _, _, kept, _, _ = solve(np.exp(mid), hk_c)
            if kept > target:
                lo = mid
            else:
                hi = mid
            if hi - lo < 2e-3:
                break
        s_H = float(np.exp(0.5 * (lo + hi)))
    else:
        s_H = float(cfg["s_H"])
    delta, mu, kept, vbm, cbm = solve(s_H)
    rec = dict(s_H=s_H, delta=float(delta), c_D=float(c_D), mu=float(mu),
               kept_fraction=kept, vbm=float(vbm), cbm=float(cbm),
               nkept=int(round(kept * kfrac.shape[0])))
    print("%-10s %s  (%.1f s)" % (name, json.dumps(rec), time.time() - t0), flush=True)
    return rec


def main(names, sub=1):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in names:
        data[name] = calibrate(name, sub)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    sub = 1
    if args and args[0].startswith("--sub="):
        sub = int(args.pop(0).split("=")[1])
    if args == ["batch"]:
        args = ["batch%02d" % j for j in range(32)]
    main(args or ["tiny3", "tiny4", "metal6", "plain8", "mixed48"], sub)
