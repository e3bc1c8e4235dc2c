"""Variant-ranking study (Sections "Matrix Multiplication", "DG
Differentiation" and "Finite Differences"; the ranking criterion of Section
"Introduction").

The paper's evaluation asks a model calibrated only on measurement kernels
to predict, and so to rank, equivalent variants of three computations: the
tiled and untiled square matmul, four DG differentiation variants (all
operands from global memory, u staged in LDS, D staged in LDS, D staged on
transposed element data; nunit = 64, nmat = 3) and the five-point stencil
with 16 x 16 and 18 x 18 work-groups.  This module

  * measures the variants (dg_variant_run) over a range of sizes, their
    work-removed twins (one per access pattern, one keeping every global
    access, one keeping none) and a set of microbenchmarks (empty launches,
    global streams, fused multiply-adds, LDS moves, barriers, the
    local/global overlap kernel), each with its exact counts
    (perf_variant_count; the microbenchmarks' counts carried over by name);
  * fits the paper's linear and overlap models (FP64, non-negative weights)
    to the measurement kernels only: no variant's own time enters a fit;
  * runs the paper's overlap analysis per variant (the variant's time against
    its all-access twin and the on-chip cost the microbenchmark rates give)
    and picks the linear model for variants whose on-chip work does not hide
    behind global traffic, the overlap model otherwise;
  * predicts every variant at every size and reports the geometric-mean
    relative error per variant (the paper's accuracy measure) and, per
    computation and size, whether the model orders the variants as measured.

Usage (GPU):  python -m paper_1904_09538_amd.variant_study measure OUT.jsonl
              python -m paper_1904_09538_amd.variant_study fit OUT.jsonl [--md PATH]
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import calibrate as C

NUNIT, NMAT = 64, 3
SIZES = {"mm": (512, 1024, 1536, 2048, 2560),
         "dg": (1 << 15, 1 << 16, 1 << 17, 1 << 18, 1 << 19),
         "fd": (2048, 4096, 6144, 8192, 10240)}
QUICK_SIZES = {"mm": (512, 1536), "dg": (1 << 15, 1 << 17), "fd": (2048, 6144)}
VARIANTS = {"mm": ("mm_pf", "mm_nopf"), "dg": ("dg_nopf", "dg_pfu", "dg_pfdm", "dg_pfdmt"),
            "fd": ("fd16", "fd18")}
FAMILY = {v: f for f, vs in VARIANTS.items() for v in vs}
# twins keeping one access pattern each (patterns shared by two variants are
# measured on one of them), plus every variant's all-access twin (7, for the
# overlap analysis) and no-access twin (0: launch and destination store only)
PATTERN_TWINS = {"mm_pf": (1, 2, 4), "mm_nopf": (1, 2), "dg_nopf": (1, 2, 4), "dg_pfu": (1, 4),
                 "dg_pfdm": (1, 2, 4), "dg_pfdmt": (1, 4), "fd16": (1, 4), "fd18": (1, 4)}
MICRO_KINDS = ("stream", "strided", "fma", "lds", "barrier", "overlap")
# cost groups of the overlap model: 0 overhead, 1 global memory, 2 on-chip
ONCHIP = ("valu_f32_sg", "lds_sg")
OVERHEAD = ("launch", "workgroups", "barrier_x_wg")
# main-space microbenchmark features and their names in the variant space
# (the microbenchmarks run every lane of every wave, so per-lane and per-wave
# counts agree)
RENAME = {"valu_f32": "valu_f32_sg", "lds_bytes": "lds_sg"}


def group_of(name):
    return 0 if name in OVERHEAD else 2 if name in ONCHIP else 1


def plan(quick=False):
    """Every launch of the study: variants, twins, microbenchmarks, empties."""
    sizes = QUICK_SIZES if quick else SIZES
    out = []
    for fam, vs in VARIANTS.items():
        for n in sizes[fam]:
            for v in vs:
                out.append({"set": "variant", "family": fam, "kind": v, "n": n})
        tw_sizes = sizes[fam][::2]
        for n in tw_sizes:
            for v in vs:
                for keep in PATTERN_TWINS[v] + (0, 5 if fam == "fd" else 7):
                    out.append({"set": "twin", "family": fam, "kind": v, "n": n, "keep": keep})
    for m in C.micro_variants(quick):
        if m["kind"] in MICRO_KINDS:
            out.append({"set": "micro", **m})
    for e in C.empty_variants(quick):
        out.append({"set": "empty", **e})
    return out


def _desc(r):
    fam, n = r["family"], r["n"]
    kw = {}
    if fam == "dg":
        kw = {"nunit": NUNIT, "nmat": NMAT}
    elif fam == "fd":
        kw = {"ld_u": n + 2, "ld_res": n}
    if r["set"] == "twin":
        kw.update(work_removed=True, keep=r["keep"])
    return kw


def measure(path, quick=False, trials=20):
    import torch

    from . import _lib

    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    flush = torch.empty(128 << 20, dtype=torch.float32, device=dev)   # 512 MB between trials
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    names = _lib.variant_feature_names()
    main_names = _lib.feature_names()
    rows = []
    t0 = time.time()

    def emit(row):
        rows.append(row)
        print(json.dumps({k: row[k] for k in row if k != "features"}), flush=True)

    todo = plan(quick)
    bufs = {}
    for fam in VARIANTS:
        mine = [r for r in todo if r.get("family") == fam and r["set"] in ("variant", "twin")]
        nmax = max(r["n"] for r in mine)
        # the largest destination of a twin whose result store is removed
        dmax = max(int(np.prod(_lib.variant_shape(r["kind"], r["n"], **_desc(r)))) for r in mine)
        if fam == "mm":
            a = torch.rand((nmax * nmax,), generator=gen, device=dev)
            b = torch.rand((nmax * nmax,), generator=gen, device=dev)
            c = torch.empty((max(nmax * nmax, dmax),), device=dev)
            bufs[fam] = (a, b, c)
        elif fam == "dg":
            u = torch.rand((nmax * NUNIT,), generator=gen, device=dev) * 2 - 1
            D = torch.rand((NMAT * NUNIT * NUNIT,), generator=gen, device=dev) * 2 - 1
            o = torch.empty((max(NMAT * nmax * NUNIT, dmax),), device=dev)
            bufs[fam] = (u, D, o)
        else:
            u = torch.rand(((nmax + 2) * (nmax + 2),), generator=gen, device=dev)
            o = torch.empty((max(nmax * nmax, dmax),), device=dev)
            bufs[fam] = (u, None, o)
    for r in todo:
        if r["set"] in ("variant", "twin"):
            kw = _desc(r)
            in0, in1, out = bufs[r["family"]]
            wgs, th = _lib.variant_shape(r["kind"], r["n"], **kw)
            if r["set"] == "twin" and not (r["keep"] & 4):
                assert out.numel() >= wgs * th, "destination buffer too small"
            tm = C.time_launch(lambda: _lib.dg_variant_run(r["kind"], r["n"], in0, in1, out, **kw), trials,
                               flush=flush)
        elif r["set"] == "empty":
            tm = C.time_launch(lambda: _lib.dg_empty_launch(r["wgs"]), trials, flush=flush)
        else:
            got = C.measure_one({k: v for k, v in r.items() if k != "set"}, trials, flush, num_cu)
            if got is None:
                continue
            tm = got["t"]
        emit({**r, "t": tm, "features": counts(r, _lib)})
    meta = {"meta": True, "device": torch.cuda.get_device_name(0), "num_cu": num_cu, "feature_names": names,
            "trials": trials, "protocol": "cold", "seconds": time.time() - t0}
    with open(path, "w") as fh:
        fh.write(json.dumps(meta) + "\n")
        for r in rows:
            fh.write(json.dumps(r) + "\n")
    return meta, rows


def counts(r, L):
    """Exact counts of a plan row in the variant feature space (host only)."""
    names = L.variant_feature_names()
    if r["set"] in ("variant", "twin"):
        return L.perf_variant_count(r["kind"], r["n"], **_desc(r)).tolist()
    main = L.feature_names()
    if r["set"] == "empty":
        c = L.perf_features_count("empty", "f32", r["wgs"])
    else:
        c = L.perf_ubench_count(r["kind"], r["n"], r["a"], r["b"], r["dtype"])
    f = {RENAME.get(k, k): int(v) for k, v in zip(main, c)}
    # the variant model has no latency term: the microbenchmarks' loop-chain
    # length is left out, every other count must have a column
    unknown = [k for k, v in f.items() if v and k not in names and k not in L.CHAIN_FEATURES]
    assert not unknown, f"microbenchmark features outside the variant space: {unknown}"
    return [f.get(k, 0) for k in names]


def _matrix(rows, cols, names):
    idx = [names.index(c) for c in cols]
    return np.array([[r["features"][i] for i in idx] for r in rows], dtype=np.float64)


def fit(path, L=None):
    """Calibrate on the measurement kernels, diagnose overlap, predict and rank
    the variants.  Returns a summary dict."""
    if L is None:
        from . import _lib as L
    meta, rows = C.load(path)
    names = meta["feature_names"]
    cal = [r for r in rows if r["set"] in ("micro", "empty", "twin")]
    tgt = [r for r in rows if r["set"] == "variant"]
    used = [k for k in names if any(r["features"][names.index(k)] for r in cal + tgt)]
    group = [group_of(k) for k in used]
    Fc, tc = _matrix(cal, used, names), np.array([r["t"]["mean"] for r in cal])
    Ft, tt = _matrix(tgt, used, names), np.array([r["t"]["mean"] for r in tgt])
    lin = L.perf_model_fit(Fc, tc, relative=True, nonneg=True)
    ovl = C.fit_overlap(L, Fc, tc, group, lin["p"], True)
    p_lin = L.perf_model_predict(Ft, lin["p"])
    p_ovl = L.perf_model_predict_overlap(Ft, group, ovl["p"], ovl["edge"])
    params = dict(zip(used, (float(x) for x in ovl["p"])))
    # the overlap analysis: variant time against its all-access twin (global
    # memory alone) and the on-chip cost at the calibrated on-chip rates
    all_twin = {(r["kind"], r["n"]): r["t"]["mean"] for r in cal
                if r["set"] == "twin" and r["keep"] == (5 if r["family"] == "fd" else 7)}
    diag = {}
    for r in tgt:
        key = (r["kind"], r["n"])
        if key not in all_twin:
            continue
        f = dict(zip(names, r["features"]))
        onchip = sum(params.get(k, 0.0) * f[k] for k in ONCHIP)
        gmem = all_twin[key]
        lo = min(gmem, onchip)
        diag.setdefault(r["kind"], []).append(
            {"n": r["n"], "t": r["t"]["mean"], "gmem_twin": gmem, "onchip_micro": onchip,
             "overlap": (gmem + onchip - r["t"]["mean"]) / lo if lo > 0 else None})
    form = {}
    for v in FAMILY:
        ov = [d["overlap"] for d in diag.get(v, []) if d["overlap"] is not None]
        form[v] = "linear" if ov and float(np.median(ov)) < 0.5 else "overlap"
    pred = np.array([p_lin[i] if form[r["kind"]] == "linear" else p_ovl[i] for i, r in enumerate(tgt)])
    per_variant = {}
    for v in FAMILY:
        ix = [i for i, r in enumerate(tgt) if r["kind"] == v]
        if not ix:
            continue
        per_variant[v] = {
            "form": form[v], "n": [tgt[i]["n"] for i in ix],
            "measured_ms": [1e3 * tt[i] for i in ix], "predicted_ms": [1e3 * pred[i] for i in ix],
            "geomean_rel_err": C.geomean(pred[ix], tt[ix]),
            "geomean_rel_err_overlap": C.geomean(p_ovl[ix], tt[ix]),
            "geomean_rel_err_linear": C.geomean(p_lin[ix], tt[ix]),
            "overlap_index_median": (float(np.median([d["overlap"] for d in diag[v] if d["overlap"] is not None]))
                                     if diag.get(v) else None)}
    rank = {}
    for fam in VARIANTS:
        ix = [i for i, r in enumerate(tgt) if r["family"] == fam]
        keys = [tgt[i]["n"] for i in ix]
        rank[fam] = C.ranking(keys, pred[ix], tt[ix])
        # per size: the measured and predicted order of the variants
        by = {}
        for i in ix:
            by.setdefault(tgt[i]["n"], []).append((tgt[i]["kind"], pred[i], tt[i]))
        rank[fam]["orders"] = {str(n): {"measured": [k for k, _, _ in sorted(v, key=lambda x: x[2])],
                                        "predicted": [k for k, _, _ in sorted(v, key=lambda x: x[1])]}
                               for n, v in sorted(by.items())}
    allr = C.ranking([(r["family"], r["n"]) for r in tgt], pred, tt)
    return {"device": meta["device"], "features": used, "groups": group, "n_calibration": len(cal),
            "n_variant_rows": len(tgt), "params_overlap": params, "edge": ovl["edge"],
            "params_linear": dict(zip(used, (float(x) for x in lin["p"]))),
            "mape_calibration_overlap": C.mape(L.perf_model_predict_overlap(Fc, group, ovl["p"], ovl["edge"]), tc),
            "per_variant": per_variant, "ranking": rank, "ranking_all": allr,
            "geomean_all": C.geomean(pred, tt), "overlap_analysis": diag}


def markdown(summary, cmd):
    """Short text summary of a fit (for a committed profile note)."""
    s = summary
    lines = [f"# Variant-ranking study ({s['device']})", "", f"Command: `{cmd}`", "",
             f"Model calibrated on {s['n_calibration']} measurement-kernel launches (microbenchmarks, empty "
             f"launches, work-removed twins); {s['n_variant_rows']} variant launches predicted, none used in "
             "the fit.", "",
             "| variant | model | geo-mean rel. error | overlap index (median) | sizes | measured ms | predicted ms |",
             "|---|---|---|---|---|---|---|"]
    for v, d in s["per_variant"].items():
        lines.append(f"| {v} | {d['form']} | {100 * d['geomean_rel_err']:.1f}% | "
                     f"{d['overlap_index_median'] if d['overlap_index_median'] is None else round(d['overlap_index_median'], 2)} | "
                     f"{', '.join(str(n) for n in d['n'])} | "
                     f"{', '.join(f'{x:.3f}' for x in d['measured_ms'])} | "
                     f"{', '.join(f'{x:.3f}' for x in d['predicted_ms'])} |")
    lines += ["", "| computation | sizes | Kendall tau (mean) | predicted fastest is fastest | regret (mean / max) |",
              "|---|---|---|---|---|"]
    for fam, r in s["ranking"].items():
        lines.append(f"| {fam} | {r['groups']} | {r['kendall_tau_mean']:.2f} | {100 * r['top1_rate']:.0f}% | "
                     f"{100 * r['regret_mean']:.1f}% / {100 * r['regret_max']:.1f}% |")
    lines += ["", "Orders per size (fastest first), measured vs predicted:", ""]
    for fam, r in s["ranking"].items():
        for n, o in r["orders"].items():
            mark = "" if o["measured"] == o["predicted"] else "  (differs)"
            lines.append(f"- {fam} {n}: {' < '.join(o['measured'])} | {' < '.join(o['predicted'])}{mark}")
    lines.append("")
    return "\n".join(lines)


def main(argv=None):
    argv = list(sys.argv[1:] if argv is None else argv)
    if not argv or argv[0] not in ("measure", "fit"):
        print(__doc__)
        return 2
    if argv[0] == "measure":
        quick = "--quick" in argv
        meta, rows = measure(argv[1], quick=quick)
        print(json.dumps({"rows": len(rows), "seconds": meta["seconds"]}))
        return 0
    s = fit(argv[1])
    print(json.dumps({k: v for k, v in s.items() if k != "overlap_analysis"}, indent=1))
    if "--md" in argv:
        path = argv[argv.index("--md") + 1]
        with open(path, "w") as fh:
            fh.write(markdown(s, "python -m paper_1904_09538_amd.variant_study measure <rows.jsonl> && "
                                 "python -m paper_1904_09538_amd.variant_study fit <rows.jsonl> --md " + path))
    return 0


if __name__ == "__main__":
    sys.exit(main())
