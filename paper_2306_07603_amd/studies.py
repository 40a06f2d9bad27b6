"""Parameter studies of arXiv:2306.07603 run through the library.

python -m paper_2306_07603_amd.studies <name> [--out FILE] [options]

  regime     Section 6.2: the flow regime (steady / periodic / quasi-periodic /
             aperiodic) of the cavities whose regime the paper reports, from the
             centre velocity and the kinetic energy of Eq. (5.1) recorded on the
             device, classified by the library's spectral classifier.
  regime_factors
             two cases the paper reports periodic, under one-factor changes of
             the readings the paper leaves open: grid nodes, time-step rule,
             central weight of Eq. (2.5).
  precision  the 257 x 257 precision sweep: steady states in FP64, and the FP32
             storage modes run as many steps, velocity error against FP64.
  lag        Step (2) with the lagged lambda of Section 3 against its implicit
             fixed point: transient difference and steady states.
  stress     a high-Reynolds stability check (theta = 45 deg, Re = 50 000).
  unsteady   the 1025 x 1025 unsteady case in FP16-deviation, FP32 and FP64
             storage: time-averaged |u| differences and throughput.
  adjoint    the 129 x 129 gradient case: discrete adjoint (FP32SRF and FP64
             trajectories), tangent sweep and central differences, timed.

Every study prints one progress line per chunk of steps and writes a JSON
summary.  Inputs are the paper's problem statement with seeded parameters; no
dataset is read.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import ifdlbm as M

# (theta, n, Re, regime the paper reports) -- Section 6.2, 256 x 256 grids
PAPER_REGIMES = [
    (60.0, 1.5, 3000.0, "steady"), (60.0, 1.5, 4000.0, "periodic"), (60.0, 1.5, 5000.0, "periodic"),
    (60.0, 1.0, 2000.0, "steady"), (60.0, 1.0, 2500.0, "periodic"), (60.0, 1.0, 3000.0, "quasi-periodic"),
    (60.0, 1.0, 4000.0, "turbulent"), (60.0, 0.5, 1000.0, "periodic"), (60.0, 0.5, 2000.0, "periodic"),
    (75.0, 1.5, 5000.0, "steady"), (75.0, 1.5, 6000.0, "periodic"),
    (45.0, 1.5, 6000.0, "quasi-periodic"), (45.0, 1.5, 7000.0, "periodic"),
]


def log(msg: str) -> None:
    print("[study] " + msg, flush=True)


def to_steady(h, tol: float, max_steps: int, chunk: int = 100000, label: str = ""):
    """ifdlbm_run_to_steady in chunks, with a progress line per chunk: returns
    (all converged, steps per cavity, E(u), E(P))."""
    total = None
    t0 = time.time()
    done = 0
    while True:
        rc, steps, ru, rp = M.ifdlbm_run_to_steady(h, tol, min(chunk, max_steps - done))
        total = steps.copy() if total is None else total + steps
        done += min(chunk, max_steps - done)
        log("%s: %d steps, E(u) max %.2e, %.0f s" % (label, done, np.nanmax(ru), time.time() - t0))
        if rc == M.IFDLBM_OK or done >= max_steps:
            return rc == M.IFDLBM_OK, total, ru, rp


def regime(n_side: int = 257, time_units: float = 3000.0, every: int = 50, precision: str = "fp32srf",
           chunk: int = 100000, steady_tol: float = 1e-4, cases=None, mix=None) -> dict:
    """Run the cases of PAPER_REGIMES (all, or the listed indices) for
    `time_units` (lid speed 0.1, height 1), record every `every` steps,
    classify the second half of the record."""
    table = [PAPER_REGIMES[i] for i in cases] if cases else PAPER_REGIMES
    cav = [M.Cavity(n_side, n_side, re, n, th, 0.1) for th, n, re, _ in table]
    o = M.ifdlbm_default_options(precision=precision, residual_every=1000, graph_steps=1000)
    if mix is not None:
        o.mix = mix
    h = M.ifdlbm_create(cav, o)
    dts = [M.ifdlbm_time_step(h, c) for c in range(len(cav))]
    steps = int(time_units / min(dts))
    cap = steps // every + 2
    M.ifdlbm_record(h, every, cap)
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        k = max(1000, k // 1000 * 1000)
        M.ifdlbm_step(h, k)
        M.ifdlbm_sync(h)
        done += k
        log("regime: %d / %d steps, %.0f s" % (done, steps, time.time() - t0))
    ru, _ = M.ifdlbm_get_residuals(h)
    out = []
    for c, (th, n, re, paper) in enumerate(table):
        st, u, v, ke = M.ifdlbm_get_record(h, c, cap)
        half = st.size // 2
        dt_sample = every * dts[c]
        rk = M.ifdlbm_classify(ke[half:], dt_sample, steady_tol) if np.all(np.isfinite(ke[half:])) else None
        rc_ = M.ifdlbm_classify(u[half:], dt_sample, steady_tol) if np.all(np.isfinite(u[half:])) else None
        out.append({"theta": th, "n": n, "re": re, "paper": paper, "status": M.ifdlbm_status(h, c),
                    "time_units": float(st[-1] * dts[c]) if st.size else 0.0,
                    "ke": rk, "u_centre": rc_, "u_last": float(u[-1]) if u.size else None,
                    "v_last": float(v[-1]) if v.size else None, "res_u_final": float(ru[c])})
        log("theta %g n %.1f Re %g: paper %s, ke %s (f %.4g, harm %.2f), u %s (f %.4g), E(u) %.1e"
            % (th, n, re, paper, rk["name"] if rk else "non-finite", rk["f_main"] if rk else 0,
               rk["harmonic_fraction"] if rk else 0, rc_["name"] if rc_ else "non-finite",
               rc_["f_main"] if rc_ else 0, ru[c]))
    return {"study": "regime", "n_side": n_side, "time_units": time_units, "every": every, "precision": precision,
            "mix": o.mix,
            "steady_tol": steady_tol, "steps": steps, "seconds": time.time() - t0, "cases": out}


# One-factor variants of the regime study: (label, nodes per side, options).  The base is the library's
# default reading (257 nodes for the paper's 256 x 256 grid, contravariant time step R11, central weight
# 0.75 of Eq. 2.5); each variant changes one of them.
REGIME_FACTORS = [
    ("base", 257, {}),
    ("256 nodes", 256, {}),
    ("Cartesian time step", 257, {"dt_rule": M.IFDLBM_DT_CARTESIAN}),
    ("central weight 0.9", 257, {"mix": 0.9}),
    ("central weight 0.5", 257, {"mix": 0.5}),
]
# the two cases the paper reports periodic where the base reading finds a steady flow
REGIME_FACTOR_CASES = [(60.0, 1.0, 2500.0), (75.0, 1.5, 6000.0)]


def regime_factors(time_units: float = 10000.0, every: int = 50, precision: str = "fp32srf",
                   chunk: int = 100000, steady_tol: float = 1e-4) -> dict:
    """The cases of REGIME_FACTOR_CASES under each variant of REGIME_FACTORS, for `time_units` each.  Variants
    with the same options share a handle; the handles step in turn, each on its own stream, so that their
    small launches overlap on the GPU.  Records and classification as in regime()."""
    groups = {}
    for label, side, opt in REGIME_FACTORS:
        key = tuple(sorted(opt.items()))
        groups.setdefault(key, []).extend((label, side, case) for case in REGIME_FACTOR_CASES)
    runs = []
    for key, members in groups.items():
        o = M.ifdlbm_default_options(precision=precision, residual_every=1000, graph_steps=1000, **dict(key))
        cav = [M.Cavity(side, side, re, n, th, 0.1) for _, side, (th, n, re) in members]
        h = M.ifdlbm_create(cav, o)
        dts = [M.ifdlbm_time_step(h, c) for c in range(len(cav))]
        steps = int(time_units / min(dts)) // 1000 * 1000 + 1000
        cap = steps // every + 2
        M.ifdlbm_record(h, every, cap)
        runs.append({"h": h, "members": members, "dts": dts, "steps": steps, "cap": cap, "done": 0,
                     "options": dict(key)})
    t0 = time.time()
    while any(r["done"] < r["steps"] for r in runs):
        for r in runs:
            k = min(chunk, r["steps"] - r["done"])
            if k > 0:
                M.ifdlbm_step(r["h"], k)
                r["done"] += k
        for r in runs:
            M.ifdlbm_sync(r["h"])
        log("regime factors: %s steps, %.0f s" % ([r["done"] for r in runs], time.time() - t0))
    out = []
    for r in runs:
        h = r["h"]
        ru, _ = M.ifdlbm_get_residuals(h)
        for c, (label, side, (th, n, re)) in enumerate(r["members"]):
            st, u, v, ke = M.ifdlbm_get_record(h, c, r["cap"])
            half = st.size // 2
            dt_sample = every * r["dts"][c]
            rk = M.ifdlbm_classify(ke[half:], dt_sample, steady_tol) if np.all(np.isfinite(ke[half:])) else None
            rc_ = M.ifdlbm_classify(u[half:], dt_sample, steady_tol) if np.all(np.isfinite(u[half:])) else None
            out.append({"variant": label, "n_side": side, "options": r["options"], "theta": th, "n": n, "re": re,
                        "dt": r["dts"][c], "time_units": float(st[-1] * r["dts"][c]) if st.size else 0.0,
                        "status": M.ifdlbm_status(h, c), "ke": rk, "u_centre": rc_, "res_u_final": float(ru[c])})
            log("%-22s theta %g n %.1f Re %g: %.0f time units, ke %s (rel amp %.2e, f %.4g), u %s (rel amp %.2e, "
                "f %.4g), E(u) %.1e"
                % (label, th, n, re, out[-1]["time_units"], rk["name"] if rk else "non-finite",
                   rk["rel_amplitude"] if rk else 0, rk["f_main"] if rk else 0, rc_["name"] if rc_ else "non-finite",
                   rc_["rel_amplitude"] if rc_ else 0, rc_["f_main"] if rc_ else 0, ru[c]))
        h.close()
    return {"study": "regime_factors", "time_units": time_units, "every": every, "precision": precision,
            "steady_tol": steady_tol, "seconds": time.time() - t0, "cases": out}


def precision(n_side: int = 257, tol: float = 1e-8, max_steps: int = 2000000,
              modes=("fp32srf", "fp32sr", "fp32", "fp32x", "fp16dev")) -> dict:
    """Steady states of Re = 1000, n in {0.5, 1, 1.5} x theta in {45, 60, 90}
    in FP64 to E(u), E(P) <= tol, then the FP32 storage modes for as many steps."""
    specs = [(th, n) for n in (0.5, 1.0, 1.5) for th in (45.0, 60.0, 90.0)]
    cav = [M.Cavity(n_side, n_side, 1000.0, n, th, 0.1) for th, n in specs]
    t0 = time.time()
    h64 = M.ifdlbm_create(cav, M.ifdlbm_default_options(precision="fp64", residual_every=1000, graph_steps=1000))
    ok, steps, ru, rp = to_steady(h64, tol, max_steps, label="precision fp64")
    log("fp64: converged %s, steps %s, %.0f s" % (ok, list(steps), time.time() - t0))
    ref = [M.ifdlbm_get_fields(h64, c) for c in range(len(cav))]
    stat = [M.ifdlbm_status(h64, c) for c in range(len(cav))]
    res = {"study": "precision", "n_side": n_side, "tol": tol, "cases": []}
    errs = {}
    for prec in modes:
        h = M.ifdlbm_create(cav, M.ifdlbm_default_options(precision=prec, residual_every=1000, graph_steps=1000))
        e = []
        # every cavity runs as many steps as its FP64 run took: step the batch to the largest count and read
        # each cavity when its count is reached
        order = np.argsort(steps)
        done = 0
        for c in order:
            M.ifdlbm_step(h, int(steps[c]) - done)
            done = int(steps[c])
            u, v, _ = M.ifdlbm_get_fields(h, int(c))
            scale = max(np.abs(ref[c][0]).max(), np.abs(ref[c][1]).max())
            e.append((int(c), float(max(np.abs(u - ref[c][0]).max(), np.abs(v - ref[c][1]).max()) / scale)))
        errs[prec] = dict(e)
        log("%s: %s, %.0f s" % (prec, ["%.1e" % errs[prec][c] for c in range(len(cav))], time.time() - t0))
    for c, (th, n) in enumerate(specs):
        res["cases"].append({"theta": th, "n": n, "re": 1000.0, "fp64_status": stat[c], "steps": int(steps[c]),
                             "res_u": float(ru[c]), "res_p": float(rp[c]),
                             "vel_error": {p: errs[p][c] for p in errs}})
    res["seconds"] = time.time() - t0
    return res


def lag(n_side: int = 65) -> dict:
    """Lagged against implicit lambda (Step 2): the velocity difference after
    a few time units, and at steady state."""
    specs = [(60.0, 0.5, 100.0), (60.0, 1.5, 100.0), (45.0, 0.75, 400.0)]
    cav = [M.Cavity(n_side, n_side, re, n, th, 0.1) for th, n, re in specs]
    out = {"study": "lag", "n_side": n_side, "cases": []}
    hl = M.ifdlbm_create(cav, M.ifdlbm_default_options(precision="fp64", residual_every=500, graph_steps=1000))
    hi = M.ifdlbm_create(cav, M.ifdlbm_default_options(precision="fp64", residual_every=500, graph_steps=1000,
                                                       lambda_mode=M.IFDLBM_LAMBDA_IMPLICIT))
    marks = []
    for n in (10, 100, 1000, 10000):
        M.ifdlbm_step(hl, n - (marks[-1] if marks else 0))
        M.ifdlbm_step(hi, n - (marks[-1] if marks else 0))
        marks.append(n)
        row = []
        for c in range(len(cav)):
            ul, vl, _ = M.ifdlbm_get_fields(hl, c)
            ui, vi, _ = M.ifdlbm_get_fields(hi, c)
            scale = max(np.abs(ul).max(), np.abs(vl).max())
            row.append(float(max(np.abs(ul - ui).max(), np.abs(vl - vi).max()) / scale))
        log("lag: step %d, relative velocity difference %s" % (n, ["%.2e" % x for x in row]))
        out.setdefault("transient", []).append({"step": n, "diff": row})
    rl = to_steady(hl, 1e-9, 3000000, label="lag lagged")
    ri = to_steady(hi, 1e-9, 3000000, label="lag implicit")
    for c, (th, n, re) in enumerate(specs):
        ul, vl, _ = M.ifdlbm_get_fields(hl, c)
        ui, vi, _ = M.ifdlbm_get_fields(hi, c)
        scale = max(np.abs(ul).max(), np.abs(vl).max())
        d = float(max(np.abs(ul - ui).max(), np.abs(vl - vi).max()) / scale)
        out["cases"].append({"theta": th, "n": n, "re": re, "steps_lagged": int(rl[1][c]),
                             "steps_implicit": int(ri[1][c]), "steady_diff": d})
        log("lag: theta %g n %g Re %g steady after %d / %d steps, difference %.2e"
            % (th, n, re, rl[1][c], ri[1][c], d))
    return out


STRESS_VARIANTS = [("mix 0.5, CFL 0.5", {"mix": 0.5}), ("central stencil (mix 1)", {"mix": 1.0}),
                   ("mix 0.75 (default)", {"mix": 0.75}), ("CFL 0.25, mix 0.5", {"cfl": 0.25, "mix": 0.5})]


def stress(n_side: int = 129, time_units: float = 500.0) -> dict:
    """theta = 45 deg, Re = 50 000 on 129 x 129 (Newtonian and two power
    laws) for `time_units`: does the run stay finite?  Repeated with the
    options the paper leaves open (the mixing weight of Eq. 2.5, the CFL)."""
    specs = [(45.0, 1.0, 50000.0), (45.0, 0.8, 50000.0), (45.0, 1.2, 50000.0)]
    cav = [M.Cavity(n_side, n_side, re, n, th, 0.1) for th, n, re in specs]
    out = {"study": "stress", "n_side": n_side, "time_units": time_units, "variants": []}
    for label, opt in STRESS_VARIANTS:
        h = M.ifdlbm_create(cav, M.ifdlbm_default_options(precision="fp64", residual_every=1000, graph_steps=1000,
                                                          **opt))
        steps = int(time_units / min(M.ifdlbm_time_step(h, c) for c in range(len(cav)))) // 1000 * 1000
        t0 = time.time()
        for k in range(0, steps, 100000):
            M.ifdlbm_step(h, min(100000, steps - k))
            M.ifdlbm_sync(h)
            log("stress %s: %d / %d steps, %.0f s" % (label, min(k + 100000, steps), steps, time.time() - t0))
        res = M.ifdlbm_get_residuals(h)
        cases = []
        for c, (th, n, re) in enumerate(specs):
            u, v, _ = M.ifdlbm_get_fields(h, c)
            finite = bool(np.all(np.isfinite(u)) and np.all(np.isfinite(v)))
            cases.append({"theta": th, "n": n, "re": re, "finite": finite, "status": M.ifdlbm_status(h, c),
                          "res_u": float(res[0][c]), "max_speed": float(np.hypot(u, v).max()) if finite else None})
            log("stress %s: theta %g n %g Re %g finite %s, E(u) %.2e"
                % (label, th, n, re, finite, res[0][c]))
        out["variants"].append({"label": label, "options": opt, "steps": steps, "cases": cases})
        h.close()
    return out


def unsteady(n_side: int = 1025, steps: int = 200000, average_from: int = 100000, every: int = 1000) -> dict:
    """theta = 75 deg, n = 1.2, Re = 1e4 on 1025 x 1025 in FP16-deviation, FP32
    (stochastic rounding, FP32 and FP64 arithmetic) and FP64 storage: time average of |u| over steps
    [average_from, steps) sampled every `every` steps, and throughput."""
    cav = [M.Cavity(n_side, n_side, 1e4, 1.2, 75.0, 0.1)]
    out = {"study": "unsteady", "n_side": n_side, "steps": steps, "average_from": average_from, "every": every,
           "runs": {}}
    means = {}
    for prec in ("fp16dev", "fp32srf", "fp32sr", "fp64"):
        h = M.ifdlbm_create(cav, M.ifdlbm_default_options(precision=prec, residual_every=1000, graph_steps=1000))
        t0 = time.time()
        acc, nacc = None, 0
        done = 0
        while done < steps:
            M.ifdlbm_step(h, every)
            done += every
            if done > average_from:
                u, v, _ = M.ifdlbm_get_fields(h, 0)
                s = np.hypot(u, v)
                acc = s if acc is None else acc + s
                nacc += 1
            if done % 20000 == 0:
                log("unsteady %s: %d / %d steps, %.0f s" % (prec, done, steps, time.time() - t0))
        M.ifdlbm_sync(h)
        wall = time.time() - t0
        means[prec] = acc / nacc
        out["runs"][prec] = {"seconds": wall, "samples": nacc,
                             "mlups_with_sampling": n_side * n_side * steps / wall / 1e6}
        h.close()
    ref = means["fp64"]
    for prec in ("fp16dev", "fp32srf", "fp32sr"):
        out["runs"][prec]["mean_speed_rel_diff_vs_fp64"] = float(np.abs(means[prec] - ref).max() / ref.max())
        log("unsteady %s: time-averaged |u| max relative difference to FP64 %.2e"
            % (prec, out["runs"][prec]["mean_speed_rel_diff_vs_fp64"]))
    return out


def adjoint(n_side: int = 129, steps: int = 20000, checkpoint_every: int = 500) -> dict:
    """Gradient of the kinetic energy (Eq. 5.1) after `steps` steps, Re 400, n 0.7,
    theta 60: the discrete adjoint (FP32SRF and FP64 trajectories), the tangent
    sweep and central differences (h = 1e-4) of the FP64 forward, with times."""
    import math
    re, n, th, u = 400.0, 0.7, 60.0, 0.1
    out = {"study": "adjoint", "n_side": n_side, "steps": steps, "checkpoint_every": checkpoint_every, "runs": {}}

    def ke(theta_deg, nn, uu):
        h = M.ifdlbm_create([M.Cavity(n_side, n_side, re, nn, theta_deg, uu)],
                            M.ifdlbm_default_options(precision="fp64", graph_steps=1000, residual_every=1000))
        M.ifdlbm_step(h, steps)
        e = M.ifdlbm_kinetic_energy(h, 0)
        h.close()
        return e

    t0 = time.time()
    hh = 1e-4
    fd = [(ke(th + math.degrees(hh), n, u) - ke(th - math.degrees(hh), n, u)) / (2 * hh),
          (ke(th, n + hh, u) - ke(th, n - hh, u)) / (2 * hh),
          (ke(th, n, u + hh * u) - ke(th, n, u - hh * u)) / (2 * hh * u)]
    out["runs"]["central_differences"] = {"grad": fd, "seconds": time.time() - t0, "forward_runs": 6}
    log("adjoint: central differences %s, %.1f s" % (["%.6e" % g for g in fd], time.time() - t0))
    cav = M.Cavity(n_side, n_side, re, n, th, u)
    for name, fn in (("adjoint_fp32srf", lambda: M.ifdlbm_adjoint(cav, M.ifdlbm_default_options(precision="fp32srf"),
                                                                     steps, checkpoint_every)),
                     ("adjoint_fp64", lambda: M.ifdlbm_adjoint(cav, M.ifdlbm_default_options(precision="fp64"),
                                                                 steps, checkpoint_every)),
                     ("tangent_fp64", lambda: M.ifdlbm_gradient(cav, M.ifdlbm_default_options(), steps))):
        t0 = time.time()
        J, g = fn()
        dt = time.time() - t0
        rel = [abs(g[q] - fd[q]) / abs(fd[q]) for q in range(3)]
        out["runs"][name] = {"J": J, "grad": [float(x) for x in g], "seconds": dt, "rel_vs_fd": rel}
        log("adjoint: %s J %.10e grad %s, rel to differences %s, %.1f s"
            % (name, J, ["%.6e" % x for x in g], ["%.1e" % r for r in rel], dt))
    return out


STUDIES = {"regime": regime, "regime_factors": regime_factors, "precision": precision, "lag": lag, "stress": stress, "unsteady": unsteady,
           "adjoint": adjoint}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("name", choices=sorted(STUDIES))
    ap.add_argument("--out", default="")
    ap.add_argument("--time-units", type=float, default=None, help="regime / stress: simulated time")
    ap.add_argument("--modes", default="", help="precision: comma-separated FP32 storage modes to compare")
    ap.add_argument("--max-steps", type=int, default=None, help="precision: step limit of the FP64 runs")
    ap.add_argument("--cases", default="", help="regime: comma-separated indices into the paper's regime table")
    ap.add_argument("--mix", type=float, default=None, help="regime: central weight of Eq. (2.5)")
    args = ap.parse_args(argv)
    kw = {}
    if args.time_units is not None and args.name in ("regime", "regime_factors", "stress"):
        kw["time_units"] = args.time_units
    if args.name == "regime" and args.cases:
        kw["cases"] = [int(x) for x in args.cases.split(",")]
    if args.name == "regime" and args.mix is not None:
        kw["mix"] = args.mix
    if args.name == "precision":
        if args.modes:
            kw["modes"] = tuple(args.modes.split(","))
        if args.max_steps:
            kw["max_steps"] = args.max_steps
    res = STUDIES[args.name](**kw)
    text = json.dumps(res, indent=1, default=float)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text[:2000])
    return 0


if __name__ == "__main__":
    sys.exit(main())
