"""Drivers for the measured workloads of the boiling convection cell.

  python -m paper_1111_0905_amd.experiments convection --n 128 --rho 1.93 --ra 1e6 --steps 20000
  python -m paper_1111_0905_amd.experiments pair --n 512 --steps 50000      (boiling vs single phase)
  python -m paper_1111_0905_amd.experiments precision --n 512 --steps 5000  (FP32 vs FP16/BF16 storage)
  python -m paper_1111_0905_amd.experiments adjoint --n 64 --steps 400      (checkpointed gradients)

Every lattice update and every diagnostic reduction runs in the HIP library;
this module only sequences calls and post-processes the returned profiles
(time series, plane averages) and, for the bubble statistics, the density
field copied to the host.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import lbm, thermo

TC = 0.08                          # walled-column linear stability ends between 0.08 and 0.1
NU = 0.0165                       # kinematic viscosity of Table 1


def cell_params(n, rho_mean, Ra, storage="fp32", T_c=TC, tau_nu=0.5 + 3 * NU, Pr=9.0,
                rho_kappa=0.5, c_v=1.0, periodic_z=0, **kw):
    """Parameters of the convection cell: T_d = 0.95 T_c, T_u = 0.85 T_c,
    tau_kappa from Pr = 9 in the liquid at the mid temperature (Table 1),
    gravity from the Rayleigh number at mid height.  The adiabatic gradient
    grows with g, so Ra has a maximum over g; a larger request is capped at
    0.7 of it (p.rayleigh holds the Ra used)."""
    G = thermo.coupling_for_tc(T_c)
    T_d, T_u = 0.95 * T_c, 0.85 * T_c
    Tm = 0.5 * (T_d + T_u)
    tau_kappa = thermo.tau_kappa_for_prandtl(Pr, (tau_nu - 0.5) / 3.0, rho_mean, Tm, G,
                                             rho_kappa, c_v)
    if Ra > 0:
        ra_max = thermo.max_rayleigh(n, rho_mean, T_d, T_u, G, tau_nu, tau_kappa, rho_kappa, c_v)
        Ra_eff = min(Ra, 0.7 * ra_max)   # beyond this the adiabatic gradient takes over
        g = thermo.gravity_for_rayleigh(Ra_eff, n, rho_mean, T_d, T_u, G, tau_nu, tau_kappa,
                                        rho_kappa, c_v)
    else:
        Ra_eff, g = 0.0, 0.0
    p = lbm.Params(n, n, n, storage=lbm.STORAGE[storage], tau_nu=tau_nu, tau_kappa=tau_kappa,
                   G=G, T_d=T_d, T_u=T_u, gravity=g, c_v=c_v, rho_kappa=rho_kappa,
                   rho_ref=rho_mean, T_ref=Tm, T_lat=Tm, periodic_z=periodic_z, **kw)
    p.rayleigh = Ra_eff
    return p


BOIL_MARGIN = 0.12


def boiling_density(n, Ra, T_c=TC, margin=BOIL_MARGIN, **kw):
    """Mean density of the boiling cell: `margin` below the mean density of
    the hydrostatic liquid column whose bottom layer sits on the liquid
    spinodal.  Once convection mixes the bulk, the bottom layer of a cell only
    slightly past that threshold stays liquid (with T_c = 0.12 at 128^3,
    Ra ~ 1e6, margins 0.045 and 0.1 formed no vapour within 10^4 steps; at
    0.12 a vapour film formed on the bottom wall and broke up into rising
    bubbles within 3 x 10^4 steps; from 0.16 on the film persisted).  With the
    cell's T_c = 0.08 and margin 0.12 a film forms within about 1.2 x 10^4
    steps at 128^3 and feeds 4-7 rising bubbles in the statistically steady
    state.  Gravity depends on the density through Ra, so the two are
    iterated to a fixed point."""
    G = thermo.coupling_for_tc(T_c)
    rho = 1.975 - margin
    for _ in range(20):
        p = cell_params(n, rho, Ra, T_c=T_c, **kw)
        new = thermo.boiling_threshold_density(n, p.T_d, p.T_u, G, p.gravity) - margin
        if abs(new - rho) < 1e-6:
            break
        rho = new
    return rho


def seeded_density(n, rho_mean, amp, seed, profile=None):
    """rho_mean (1 + amp (2u - 1)) per node, u seeded uniform; with a
    vertical profile rho(z) of mean rho_mean the field is scaled plane by
    plane to it (the same noise either way)."""
    import synth
    r = synth.noisy_density(n, n, n, rho_mean, amp, seed)
    if profile is not None:
        r *= (np.asarray(profile) / rho_mean).reshape(n, 1, 1)
    return torch.from_numpy(r).cuda().reshape(-1)


def initial_temperature(p, n, amp, seed):
    """Conduction profile plus seeded noise of amp (T_d - T_u) (2u - 1) per
    node (seed + 1 so it is independent of the density noise): without a
    temperature perturbation the convective instability of a quiet liquid
    grows only from the density noise, over many free-fall times."""
    import synth
    k = np.arange(n, dtype=np.float64)
    Tz = p.T_d + (p.T_u - p.T_d) * (k + 0.5) / n
    u = synth.noisy_density(n, n, n, 1.0, 1.0, seed + 1) - 1.0
    T = Tz.reshape(n, 1, 1) + amp * (p.T_d - p.T_u) * u
    return torch.from_numpy(T).cuda().reshape(-1)


def initial_density(p, n, rho_mean, amp, seed):
    """Seeded field on the hydrostatic liquid column when one exists (a
    uniform start would launch a pressure wave of amplitude g rho L, which
    the weakly damped liquid at tau_nu = 0.5495 does not survive at
    rho = 2.49); uniform mean density otherwise (the boiling cell, whose
    bottom layer has no liquid state)."""
    prof = thermo.hydrostatic_profile(n, rho_mean, p.T_d, p.T_u, p.G, p.gravity)
    return seeded_density(n, rho_mean, amp, seed, prof), prof is not None


FLUX_RANGE = 400.0      # heat-flux pdf range, +- in units of the diffusive flux kappa dT / L
FLUX_BINS = 800


def convection(p: lbm.Params, rho0, steps: int, diag_every: int, log=None, phase_every=0,
               T0=None):
    """Run and record Nu_bot, Nu_top, the bulk-averaged Nu(z), the vapour
    fraction and the density minimum every diag_every steps, and the bubble
    statistics every phase_every steps (0: only at the end).  Over the second
    half of the run the bulk heat flux rho U v_z is histogrammed at every
    record (the pdf of Fig. 2, bottom inset).  Returns the record."""
    lat = lbm.Lattice(p, rho0, T0)
    tot0 = lat.moments()
    rec = {"t": [], "nu_bot": [], "nu_top": [], "nu_bulk": [], "mass_drift": [],
           "vapour_fraction": [], "rho_min": [], "phases_t": [], "ok": True}
    n = p.nz
    bulk = slice(n // 4, 3 * n // 4)
    q_unit = thermo.kappa(p.tau_kappa, p.rho_kappa, p.c_v) * (p.T_d - p.T_u) / n
    flux_counts = np.zeros(FLUX_BINS, dtype=np.int64)
    flux_sums = np.zeros(5)
    flux_oor = 0
    step_ms = 0.0
    t = 0
    while t < steps:
        k = min(diag_every, steps - t)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.h.stream)
        lat.step(k)
        e1.record(lat.h.stream)
        torch.cuda.synchronize()
        step_ms += e0.elapsed_time(e1)
        t += k
        try:
            tot = lat.moments()
        except lbm.LbmError as e:
            rec["ok"] = False
            rec["error"] = str(e)
            break
        nb, nt, nu_z, T_z = lat.nusselt()
        rec["t"].append(t)
        rec["nu_bot"].append(nb)
        rec["nu_top"].append(nt)
        rec["nu_bulk"].append(float(np.mean(nu_z[bulk])))
        rec["mass_drift"].append(float(tot[0] / tot0[0] - 1))
        if 2 * t > steps:
            c, o, sm = lat.histogram(n // 4, 3 * n // 4, lbm.LBM_Q_HEATFLUX,
                                     (-FLUX_RANGE * q_unit, FLUX_RANGE * q_unit), FLUX_BINS)
            flux_counts += c.cpu().numpy().ravel()
            flux_oor += o
            flux_sums += sm
        _, fl = lat.fields()
        rec["vapour_fraction"].append(float((fl[0] < 1.0).double().mean()))
        rec["rho_min"].append(float(fl[0].min()))
        del fl
        if phase_every and t % phase_every == 0:
            ph = phase_statistics(lat)
            vols = ph.pop("bubble_volumes")
            ph.update(t=t, max_volume=max(vols, default=0),
                      mean_volume=float(np.mean(vols)) if vols else 0.0)
            rec["phases_t"].append(ph)
            if log:
                print(json.dumps({"phases": ph}), file=log, flush=True)
        if log:
            print(json.dumps({"t": t, "nu_bot": round(nb, 4), "nu_top": round(nt, 4),
                              "nu_bulk": round(rec["nu_bulk"][-1], 4),
                              "vap": round(rec["vapour_fraction"][-1], 5),
                              "rho_min": round(rec["rho_min"][-1], 4)}), file=log, flush=True)
    if rec["ok"]:
        nb, nt, nu_z, T_z = lat.nusselt()
        rec["T_z"] = [float(x) for x in T_z]
        rec["nu_z"] = [float(x) for x in nu_z]
        if flux_sums[0] > 0:
            mean = flux_sums[1] / flux_sums[0]
            rec["bulk_flux_pdf"] = {
                "unit": "kappa (T_d - T_u) / L", "range": [-FLUX_RANGE, FLUX_RANGE],
                "counts": flux_counts.tolist(), "out_of_range": int(flux_oor),
                "mean": mean / q_unit,
                "std": math.sqrt(max(flux_sums[2] / flux_sums[0] - mean * mean, 0.0)) / q_unit,
                "samples": int(flux_sums[0])}
        rec["rho_T_hist"] = rho_T_histograms(lat, p)
        rmax = min(128, p.nx // 2, p.ny // 2)
        rec["structure"] = {}
        for name, q in (("vz", lbm.LBM_Q_VZ), ("T", lbm.LBM_Q_T)):
            s2, s4 = lat.structure_functions(n // 4, 3 * n // 4, q, rmax)
            rec["structure"][name] = {"S2": s2.tolist(), "S4": s4.tolist(),
                                      "flatness": (s4 / np.maximum(s2, 1e-300) ** 2).tolist()}
    rec["ms_per_step"] = step_ms / max(t, 1)
    rec["mlups"] = p.n / (rec["ms_per_step"] * 1e-3) / 1e6
    rec["lattice"] = lat
    return rec


def rho_T_histograms(lat, p, rho_bins=150, T_bins=100):
    """Joint (rho, T) histograms of the bottom (k < L/8), bulk (L/4 <= k <
    3L/4) and top (k >= 7L/8) regions (Fig. 2, top panel): rho in [0, 3],
    T in [0.8, 1.0] T_c; counts as nested lists [rho bin][T bin]."""
    n = p.nz
    Tc = -p.G / math.e ** 2
    out = {"rho_range": [0.0, 3.0], "T_range": [0.8 * Tc, 1.0 * Tc]}
    for name, (k0, k1) in (("bottom", (0, n // 8)), ("bulk", (n // 4, 3 * n // 4)),
                           ("top", (n - n // 8, n))):
        c, o, _ = lat.histogram(k0, k1, lbm.LBM_Q_RHO, (0.0, 3.0), rho_bins, lbm.LBM_Q_T,
                                (0.8 * Tc, 1.0 * Tc), T_bins)
        out[name] = {"counts": c.cpu().numpy().tolist(), "out_of_range": int(o)}
    return out


def bulk_slope(T_z):
    """Least-squares slope of the mean temperature over L/4 <= k < 3L/4."""
    T_z = np.asarray(T_z)
    n = len(T_z)
    k = np.arange(n // 4, 3 * n // 4)
    return float(np.polyfit(k, T_z[k], 1)[0])


def profile_asymmetry(T_z, T_d, T_u):
    """(T_centre - T_mean) / T_mean of the horizontal-mean profile (Fig. 2
    inset; the paper quotes 1 % for boiling)."""
    T_z = np.asarray(T_z)
    n = len(T_z)
    Tc = 0.5 * (T_z[n // 2 - 1] + T_z[n // 2]) if n % 2 == 0 else T_z[n // 2]
    Tm = 0.5 * (T_d + T_u)
    return float((Tc - Tm) / Tm)


def phase_statistics(lat, bins=200):
    """Density histogram peaks (vapour, liquid) and bubble volumes: 6-connected
    components of rho < (rho_g + rho_l)/2, periodic in x and y."""
    from scipy import ndimage
    _, fields = lat.fields()
    rho = fields[0].cpu().numpy()
    hist, edges = np.histogram(rho, bins=bins)
    centres = 0.5 * (edges[1:] + edges[:-1])
    split = np.searchsorted(centres, 1.0)
    rho_g = float(centres[np.argmax(hist[:split])]) if split > 0 and hist[:split].sum() > 0 else float("nan")
    rho_l = float(centres[split + np.argmax(hist[split:])])
    thr = 0.5 * (rho_g + rho_l) if math.isfinite(rho_g) else 1.0
    mask = rho < thr
    lab, nlab = ndimage.label(mask)
    if nlab > 0:
        # merge labels across the periodic x and y faces
        parent = np.arange(nlab + 1)

        def find(a):
            while parent[a] != a:
                parent[a] = parent[parent[a]]
                a = parent[a]
            return a

        for a, b in ((lab[:, :, 0], lab[:, :, -1]), (lab[:, 0, :], lab[:, -1, :])):
            m = (a > 0) & (b > 0)
            for x, y in zip(a[m].ravel(), b[m].ravel()):
                rx, ry = find(x), find(y)
                if rx != ry:
                    parent[max(rx, ry)] = min(rx, ry)
        roots = np.array([find(i) for i in range(nlab + 1)])
        vols = np.bincount(roots[lab.ravel()], minlength=nlab + 1)[1:]
        vols = vols[vols > 0]
    else:
        vols = np.zeros(0, dtype=np.int64)
    return {"rho_g": rho_g, "rho_l": rho_l, "vapour_fraction": float(mask.mean()),
            "n_bubbles": int(len(vols)), "bubble_volumes": sorted(int(v) for v in vols)}


def _summary(rec, p):
    nb = np.asarray(rec["nu_bulk"])
    half = len(nb) // 2
    out = {k: v for k, v in rec.items() if k != "lattice"}
    if len(nb):
        out["nu_bulk_mean_2nd_half"] = float(nb[half:].mean())
        out["nu_bulk_std_2nd_half"] = float(nb[half:].std())
        out["nu_bot_mean_2nd_half"] = float(np.mean(rec["nu_bot"][half:]))
        out["nu_top_mean_2nd_half"] = float(np.mean(rec["nu_top"][half:]))
    if "T_z" in rec:
        out["T_centre_minus_mean_rel"] = profile_asymmetry(rec["T_z"], p.T_d, p.T_u)
        Tm = 0.5 * (p.T_d + p.T_u)
        rho = p.rho_ref
        out["bulk_dTdz"] = bulk_slope(rec["T_z"])
        out["adiabatic_dTdz"] = -thermo.beta(rho, Tm, p.G) * Tm * p.gravity / thermo.cp(rho, Tm, p.G, p.c_v)
        out["conductive_dTdz"] = -(p.T_d - p.T_u) / p.nz
    out["params"] = {f: getattr(p, f) for f in ("nx", "ny", "nz", "storage", "tau_nu", "tau_kappa",
                                                 "G", "T_d", "T_u", "gravity", "c_v", "rho_kappa")}
    out["params"]["rayleigh"] = getattr(p, "rayleigh", None)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["convection", "pair", "precision", "adjoint"])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--rho", type=float, default=None,
                    help="mean density of the boiling cell (default: from the hydrostatic column)")
    ap.add_argument("--rho-single", type=float, default=2.49)
    ap.add_argument("--ra", type=float, default=1e6)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--diag", type=int, default=500)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--noise", type=float, default=0.01)
    ap.add_argument("--tnoise", type=float, default=0.05,
                    help="temperature noise in units of T_d - T_u (0: the plain conduction profile)")
    ap.add_argument("--ckpt", type=int, default=20)
    ap.add_argument("--margin", type=float, default=BOIL_MARGIN)
    ap.add_argument("--phase-every", type=int, default=0,
                    help="steps between bubble statistics (0: only at the end)")
    ap.add_argument("--tc", type=float, default=TC)
    ap.add_argument("--rho-wall-d", type=float, default=0.0,
                    help="wall density of the bottom wall's psi ghost (wetting); 0 = neutral")
    ap.add_argument("--rho-wall-u", type=float, default=0.0,
                    help="the same for the top wall")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    walls = dict(rho_wall_d=a.rho_wall_d, rho_wall_u=a.rho_wall_u)
    lbm.load_library()
    res = {}
    log = sys.stderr
    if a.rho is None:
        a.rho = boiling_density(a.n, a.ra, T_c=a.tc, margin=a.margin)
    if a.what == "convection":
        p = cell_params(a.n, a.rho, a.ra, a.storage, T_c=a.tc, **walls)
        rho0, hydro = initial_density(p, a.n, a.rho, a.noise, a.seed)
        T0 = initial_temperature(p, a.n, a.tnoise, a.seed) if a.tnoise > 0 else None
        rec = convection(p, rho0, a.steps, a.diag, log, a.phase_every, T0)
        res = _summary(rec, p)
        res["hydrostatic_start"] = hydro
        if rec["ok"]:
            res["phases"] = phase_statistics(rec["lattice"])
    elif a.what == "pair":
        for name, rho in (("boiling", a.rho), ("single_phase", a.rho_single)):
            p = cell_params(a.n, rho, a.ra, a.storage, T_c=a.tc, **walls)
            rho0, _ = initial_density(p, a.n, rho, a.noise, a.seed)
            T0 = initial_temperature(p, a.n, a.tnoise, a.seed) if a.tnoise > 0 else None
            rec = convection(p, rho0, a.steps, a.diag, log, a.phase_every, T0)
            res[name] = _summary(rec, p)
            if rec["ok"]:
                res[name]["phases"] = phase_statistics(rec["lattice"])
            del rec
            torch.cuda.empty_cache()
    elif a.what == "precision":
        for st in ("fp32", "fp16dev", "bf16dev"):
            p = cell_params(a.n, a.rho, a.ra, st, T_c=a.tc, **walls)
            rho0, _ = initial_density(p, a.n, a.rho, a.noise, a.seed)
            T0 = initial_temperature(p, a.n, a.tnoise, a.seed) if a.tnoise > 0 else None
            rec = convection(p, rho0, a.steps, a.diag, log, a.phase_every, T0)
            res[st] = _summary(rec, p)
            if rec["ok"]:
                res[st]["phases"] = phase_statistics(rec["lattice"])
            del rec
            torch.cuda.empty_cache()
        if all(res[s].get("ok") for s in res):
            ref = np.asarray(res["fp32"]["nu_bulk"])
            for st in ("fp16dev", "bf16dev"):
                x = np.asarray(res[st]["nu_bulk"])
                res[st]["nu_bulk_max_abs_diff_vs_fp32"] = float(np.abs(x - ref).max())
    elif a.what == "adjoint":
        from dataclasses import replace

        from . import adjoint
        import synth
        out = {}
        d = torch.from_numpy(synth.random_unit_field(a.n, a.n, a.n, 7)).cuda().reshape(-1)
        for st in ("fp32", "fp64"):
            p = cell_params(a.n, a.rho, a.ra, st, T_c=a.tc, **walls)
            rho0 = seeded_density(a.n, a.rho, a.noise, a.seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            J, dr, dTd, dG = adjoint.heat_flux_gradients(p, rho0, a.steps, a.ckpt)
            torch.cuda.synchronize()
            out[st] = {"J": J, "dJ_dTd": dTd, "dJ_dG": dG, "dJ_drho0_dir": float((dr * d).sum()),
                       "seconds": time.perf_counter() - t0}
            print(json.dumps({st: out[st]}), file=log, flush=True)
        for k in ("dJ_dTd", "dJ_dG", "dJ_drho0_dir"):
            out[f"fp32_vs_fp64_rel_{k}"] = abs(out["fp32"][k] / out["fp64"][k] - 1)
        # central differences of the FP64 forward, initial T profile held fixed
        p = cell_params(a.n, a.rho, a.ra, "fp64", T_c=a.tc)
        rho0 = seeded_density(a.n, a.rho, a.noise, a.seed)
        T0 = adjoint.conduction_profile(p)

        def J_of(q, r):
            return adjoint.heat_flux_objective(q, r, a.steps, T0)

        h = 1e-4 * p.T_d
        fd_Td = (J_of(replace(p, T_d=p.T_d + h), rho0) - J_of(replace(p, T_d=p.T_d - h), rho0)) / (2 * h)
        h = 1e-4 * abs(p.G)
        fd_G = (J_of(replace(p, G=p.G + h), rho0) - J_of(replace(p, G=p.G - h), rho0)) / (2 * h)
        h = 1e-4 * float(rho0.abs().max())
        fd_r = (J_of(p, rho0 + h * d) - J_of(p, rho0 - h * d)) / (2 * h)
        out["fd_fp64"] = {"dJ_dTd": fd_Td, "dJ_dG": fd_G, "dJ_drho0_dir": fd_r}
        for st in ("fp64", "fp32"):
            for k in ("dJ_dTd", "dJ_dG", "dJ_drho0_dir"):
                out[f"{st}_vs_fd_rel_{k}"] = abs(out[st][k] / out["fd_fp64"][k] - 1)
        out["params"] = {"n": a.n, "steps": a.steps, "ckpt": a.ckpt, "rho_mean": a.rho,
                         "gravity": p.gravity, "G": p.G, "T_d": p.T_d, "T_u": p.T_u,
                         "tau_nu": p.tau_nu, "tau_kappa": p.tau_kappa}
        res = out
    js = json.dumps(res)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(js)
    print(js[:2000])
    if res.get("ok") is False:
        sys.exit(3)


if __name__ == "__main__":
    main()
