"""Time-step error scaling of the explicit methods with full and extrapolated
demagnetizing fields (the protocol of Sec. III, Fig. 2 and Fig. 3).

For each method a reference run with a short fixed step (10 fs) and full
evaluation of Eq. (2) at every stage is compared with runs at longer fixed
steps (controller off), with full evaluation and with Eq. (6) extrapolation of
the given orders.  Every run records the mesh-averaged magnetization <M> at a
fixed sampling interval, and the error of a run is Eq. (7) over those
samples:

    eps = (1/N) sum_i |<M>_i - <M~>_i| / Ms

(with the per-cell reading of Eq. (7), the map at the end of the window, also
reported).  All runs start from the same state at t = 0 and go through the
library; the harness only drives it and compares the recorded series.

    python -m paper_2107_06729_amd.scaling --method RKF56 --p 1 2 3 4 5

prints one JSON object per (method, mode, h).
"""

import argparse
import json
import math


def eq7_series(mavg, mavg_ref, Ms):
    """Eq. (7) over rows of <M> (N x 3): mean Euclidean distance over Ms."""
    import numpy as np
    a = np.asarray(mavg, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(mavg_ref, dtype=np.float64).reshape(-1, 3)
    if len(a) != len(b):
        raise ValueError(f"series of different length ({len(a)} vs {len(b)})")
    return float(np.linalg.norm(a - b, axis=1).mean() / Ms)


def eq7_map(M, M_ref, Ms):
    """Eq. (7) over the cells of two magnetization maps (3 x cells)."""
    import numpy as np
    d = np.asarray(M, dtype=np.float64).reshape(3, -1) - np.asarray(M_ref, dtype=np.float64).reshape(3, -1)
    return float(np.sqrt((d * d).sum(axis=0)).mean() / Ms)


def _run(problem, M0, method, h, extrap, window, sample_dt, precision, tensor, stream):
    import torch
    from . import Sim, make_stepper
    s = Sim(problem, precision, stream=stream)
    if tensor is None:
        s.precompute_demag()
    else:
        s.set_demag_tensor(tensor)
    dt = torch.float32 if precision == "f32" else torch.float64
    s.set_m(torch.as_tensor(M0, dtype=dt, device="cuda:0"))
    st = make_stepper(method, extrap=extrap, h=h, adaptive=False)
    mavg = s.run(st, window, sample_dt)
    M = s.get_m().double().cpu().numpy()
    stats = s.counters()
    s.close()
    return mavg, M, stats


def error_scaling(problem, M0, method, hs, extraps=("matched",), h_ref=10e-15, window=20e-12, sample_dt=1e-12,
                  precision="f64", tensor=None, stream=None, reference=None):
    """Eq. (7) errors of `method` at the fixed steps `hs` against a reference
    run at h_ref with full evaluation.  extraps: None (full evaluation), an
    order p, or "matched"; the full-evaluation runs are always included.
    Every h must divide sample_dt and window (the samples land on steps).

    Returns a list of dicts {method, mode, p, h, eps_series, eps_map, exact,
    extrap} and the reference (mavg, M) for reuse."""
    for h in list(hs) + [h_ref]:
        k = sample_dt / h
        if abs(k - round(k)) > 1e-9 * k or abs(window / h - round(window / h)) > 1e-9 * window / h:
            raise ValueError(f"step {h} does not divide the sampling interval and the window")
    Ms = problem["Ms"]
    if reference is None:
        reference = _run(problem, M0, method, h_ref, None, window, sample_dt, precision, tensor, stream)[:2]
    mref, Mref = reference
    modes = [None] + [e for e in extraps if e is not None]
    rows = []
    for mode in modes:
        for h in hs:
            mavg, M, stats = _run(problem, M0, method, h, mode, window, sample_dt, precision, tensor, stream)
            rows.append({"method": method, "mode": "full" if mode is None else ("matched" if mode == "matched"
                                                                                 else f"p{mode}"),
                         "p": mode, "h": h, "eps_series": eq7_series(mavg, mref, Ms),
                         "eps_map": eq7_map(M, Mref, Ms), "exact": stats["exact"], "extrap": stats["extrap"]})
    return rows, reference


def observed_order(rows, mode):
    """Least-squares slope of log eps_series against log h for one mode."""
    pts = [(math.log(r["h"]), math.log(r["eps_series"])) for r in rows if r["mode"] == mode and r["eps_series"] > 0]
    n = len(pts)
    if n < 2:
        return float("nan")
    mx = sum(x for x, _ in pts) / n
    my = sum(y for _, y in pts) / n
    return sum((x - mx) * (y - my) for x, y in pts) / sum((x - mx) ** 2 for x, _ in pts)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--method", default="RKF56")
    ap.add_argument("--p", nargs="*", default=["matched"], help="extrapolation orders (or 'matched')")
    ap.add_argument("--h", nargs="*", type=float, default=[100e-15, 125e-15, 200e-15, 250e-15, 500e-15])
    ap.add_argument("--window", type=float, default=20e-12)
    ap.add_argument("--precision", default="f64")
    args = ap.parse_args()
    import workloads
    prob = workloads.FILM_256x64x1
    M0 = workloads.uniform_m(prob["n"], prob["Ms"], workloads.FILM_256x64x1_DIR)
    extraps = [e if e == "matched" else int(e) for e in args.p]
    rows, _ = error_scaling(prob, M0, args.method, args.h, extraps, window=args.window, precision=args.precision)
    for r in rows:
        print(json.dumps(r))
    for mode in sorted({r["mode"] for r in rows}):
        print(json.dumps({"mode": mode, "observed_order": observed_order(rows, mode)}))


if __name__ == "__main__":
    main()
