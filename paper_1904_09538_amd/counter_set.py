"""Hardware-counter variant set: launches every hot-path kernel at its
workload sizes under rocprofv3 --pmc, and summarises the counters beside the
library's counted features (Section "Gathering Kernel Statistics": the
counts are exact operation counts of the documented schedule; the counters
are what the GPU executed).

    python -m paper_1904_09538_amd.counter_set run --out DIR/variants.json
        Launches each variant twice between marker launches (an empty kernel
        of MARKER_WGS work-groups) and writes the variant list with the launch
        shapes the library resolved on this device.  Run it under
        rocprofv3 --pmc <counters> --output-format csv -d DIR/<pass> -- python -m ...

    python -m paper_1904_09538_amd.counter_set summarise --variants DIR/variants.json \
            --pmc DIR/pass1 DIR/pass2 ... --json profiles/counters.json --md profiles/counters_vs_features.md
        Matches the dispatches of each pass to the variants (by the markers),
        keeps the library's kernels (and, for the copy probe, every kernel),
        and writes per-variant counters per call with the counted features.

Counters used (gfx950, rocprofiler-sdk names):
  SQ_WAVES; SQ_INSTS_VALU_MFMA_MOPS_{F32,F64,BF16,F8} (matrix-core operations
  / 512); SQ_INSTS_LDS_{LOAD,STORE}_BANDWIDTH (LDS bytes of the executing
  lanes / 64); SQ_INSTS_LDS; SQ_INSTS_VMEM_{RD,WR}; SQ_INSTS_VALU_FLOPS_FP32;
  FETCH_SIZE, WRITE_SIZE (KiB between L2 and memory; each pass alone).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MARKER_WGS = 7          # work-groups of the marker launch (an empty kernel)
CALLS = 2               # measured calls per variant
PASSES = {
    "sq_mfma": "SQ_WAVES SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_BF16",
    "sq_lds": "SQ_INSTS_VALU_MFMA_MOPS_F8 SQ_INSTS_LDS_LOAD_BANDWIDTH SQ_INSTS_LDS_STORE_BANDWIDTH SQ_INSTS_LDS",
    "sq_vmem": "SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_SALU",
    "fetch": "FETCH_SIZE",
    "write": "WRITE_SIZE",
}

# (id, kind, parameters).  Sizes are the measured workloads; the extra DG
# shapes exercise the non-default schedule branches (two column blocks per
# wave, several operator groups re-reading elements from L2, FP64).
VARIANTS = [
    ("copy_1GiB", "copy", {"bytes": 1 << 30}),
    ("dg_f32_p2_2e21", "dg", {"dtype": "f32", "p": 2, "E": 1 << 21}),
    ("dg_f32_p3_2e21", "dg", {"dtype": "f32", "p": 3, "E": 1 << 21}),
    ("dg_f32_p4_2e21", "dg", {"dtype": "f32", "p": 4, "E": 1 << 21}),
    ("dg_f32_p5_2e21", "dg", {"dtype": "f32", "p": 5, "E": 1 << 21}),
    ("dg_f32_p3_2e18_epw32_w4", "dg", {"dtype": "f32", "p": 3, "E": 1 << 18,
                                        "tile": {"elems_per_wave": 32, "waves": 4}}),
    ("dg_f32_p4_2e18_panels8", "dg", {"dtype": "f32", "p": 4, "E": 1 << 18, "tile": {"d_panels": 8}}),
    ("dg_f32_p2_100003", "dg", {"dtype": "f32", "p": 2, "E": 100003}),
    ("dg_f64_p3_4096", "dg", {"dtype": "f64", "p": 3, "E": 4096}),
    ("dg_bf16_p5_2e20", "dg", {"dtype": "bf16", "p": 5, "E": 1 << 20}),
    ("dg_fp8_p5_2e20", "dg", {"dtype": "fp8", "p": 5, "E": 1 << 20}),
    ("dg_bf16_p5_2e20_ldspanels", "dg", {"dtype": "bf16", "p": 5, "E": 1 << 20, "tile": {"flags": 8}}),
    ("dg_fp8_p5_2e20_ldspanels", "dg", {"dtype": "fp8", "p": 5, "E": 1 << 20, "tile": {"flags": 8}}),
    ("dg_bf16_p5_100003_split", "dg", {"dtype": "bf16", "p": 5, "E": 100003,
                                       "tile": {"waves": 9, "d_panels": 9}}),
    ("dg_fp8native_p5_2e20", "dg", {"dtype": "fp8", "p": 5, "E": 1 << 20, "tile": {"flags": 2}}),
    # the staged body with fewer operators (fewer groups re-reading each
    # element tile from L2), and with grids of several rounds of work-groups
    ("dg_bf16_p5_2e20_nmat1", "dg", {"dtype": "bf16", "p": 5, "E": 1 << 20, "nmat": 1}),
    ("dg_bf16_p5_2e20_nmat2", "dg", {"dtype": "bf16", "p": 5, "E": 1 << 20, "nmat": 2}),
    ("dg_fp8_p5_2e20_nmat1", "dg", {"dtype": "fp8", "p": 5, "E": 1 << 20, "nmat": 1}),
    ("dg_fp8_p5_2e20_nmat2", "dg", {"dtype": "fp8", "p": 5, "E": 1 << 20, "nmat": 2}),
    ("dg_bf16_p5_2e20_grid8", "dg", {"dtype": "bf16", "p": 5, "E": 1 << 20, "tile": {"groups_per_cu": 8}}),
    ("dg_bf16_p5_2e20_grid24", "dg", {"dtype": "bf16", "p": 5, "E": 1 << 20, "tile": {"groups_per_cu": 24}}),
    ("quant_fp8_rows_2e20x216", "quant", {"to": "fp8", "rows": 1 << 20, "cols": 216}),
    ("quant_bf16_2e20x216", "quant", {"to": "bf16", "rows": 1 << 20, "cols": 216}),
    ("batched_p1_7_2e20", "batched", {"E": 1 << 20}),
    ("adjoint_p4_2e19", "adjoint", {"p": 4, "E": 1 << 19}),
    ("stencil_16384", "stencil", {"n": 16384}),
    ("stencil_1030", "stencil", {"n": 1030}),
    ("matmul_8192", "matmul", {"n": 8192}),
    ("matmul_1000", "matmul", {"n": 1000}),
    ("empty_1024", "empty", {"wgs": 1024}),
]


def _log(*a):
    print("counter_set:", *a, flush=True)


# ------------------------------------------------------------------ run (GPU)

def _dg_inputs(torch, I, dtype, p, E, dev, L):
    import numpy as np
    n = I.nunit_of_order(p)
    D = torch.from_numpy(I.gll_dmats(p)).to(dev, torch.float64 if dtype == "f64" else torch.float32)
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    u = torch.rand((E, n), generator=g, device=dev, dtype=torch.float32) * 2 - 1
    if dtype == "f64":
        u = u.double()
    extra = {}
    if dtype in ("bf16", "fp8"):
        to = "bf16" if dtype == "bf16" else "e4m3"
        qD, isD = L.dgdiff_quantize(D.reshape(3, n * n), to, per_row=True)
        qu, isu = L.dgdiff_quantize(u, to, per_row=True)
        D, u = qD.view(3, n, n), qu
        if dtype == "fp8":
            extra = {"inv_sD": isD, "inv_su": isu}
    del np
    return D, u, n, extra


def run(out_path):
    import numpy as np
    import torch

    from paper_1904_09538_amd import _lib as L, inputs as I

    dev = torch.device("cuda:0")
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    L.lib()
    recs = []
    for vid, kind, prm in VARIANTS:
        _log(f"variant {vid}")
        rec = {"id": vid, "kind": kind, "params": prm, "num_cu": num_cu}
        if kind == "copy":
            src = torch.ones(prm["bytes"] // 4, device=dev)
            dst = torch.empty_like(src)
            fn = lambda: dst.copy_(src)  # noqa: E731
            keep = (src, dst)
        elif kind == "dg":
            D, u, n, extra = _dg_inputs(torch, I, prm["dtype"], prm["p"], prm["E"], dev, L)
            M = prm.get("nmat", 3)
            if M < 3:
                D = D[:M].contiguous()
                if extra:
                    extra = {"inv_sD": extra["inv_sD"][:M].contiguous(), "inv_su": extra["inv_su"]}
            tile = L.resolve_tile(prm["dtype"], M, prm["E"], n, prm.get("tile"))
            rec["tile"] = tile
            rec["nunit"] = n
            out = torch.empty((M, prm["E"], n), device=dev,
                              dtype=torch.float64 if prm["dtype"] == "f64" else torch.float32)
            fn = lambda: L.dgdiff_apply(D, u, out=out, tile=tile, **extra)  # noqa: E731
            keep = (D, u, out, extra)
        elif kind == "quant":
            x = torch.rand((prm["rows"], prm["cols"]), device=dev) * 2 - 1
            fn = lambda: L.dgdiff_quantize(x, prm["to"] if prm["to"] == "bf16" else "e4m3", per_row=True)  # noqa: E731
            keep = (x,)
        elif kind == "batched":
            order = I.batched_orders(prm["E"])
            plan = L.BatchedPlan(order)
            Ds = {p: torch.from_numpy(I.gll_dmats(p)).float().to(dev) for p in range(1, 8)}
            u = torch.rand(plan.total, device=dev) * 2 - 1
            o = torch.empty((3, plan.total), device=dev)
            rec["plan"] = {p: plan.info(p) for p in range(1, 8)}
            rec["orders"] = {p: int((order == p).sum()) for p in range(1, 8)}
            fn = lambda: plan.apply(Ds, u, out=o)  # noqa: E731
            keep = (plan, Ds, u, o)
        elif kind == "adjoint":
            n = I.nunit_of_order(prm["p"])
            D = torch.from_numpy(I.gll_dmats(prm["p"])).float().to(dev)
            u = torch.rand((prm["E"], n), device=dev) * 2 - 1
            gr = torch.randn((3, prm["E"], n), device=dev)
            rec["nunit"] = n
            rec["tiles_bwd"] = L.resolve_backward("f32", 3, prm["E"], n)
            rec["workspace_bytes"] = int(L.lib().dgdiff_backward_workspace(L.DG_F32, 3, prm["E"], n))
            fn = lambda: L.dgdiff_backward(D, u, gr)  # noqa: E731
            keep = (D, u, gr)
        elif kind == "stencil":
            n = prm["n"]
            ld = ((n + 2 + 63) // 64) * 64
            ug = torch.rand((n + 2, ld), device=dev)
            r = torch.empty((n, n), device=dev)
            fn = lambda: L.stencil5_apply(ug, res=r, n=n)  # noqa: E731
            keep = (ug, r)
        elif kind == "matmul":
            n = prm["n"]
            a = torch.randn((n, n), device=dev)
            b = torch.randn((n, n), device=dev)
            c = torch.empty((n, n), device=dev)
            fn = lambda: L.matmul_apply(a, b, c)  # noqa: E731
            keep = (a, b, c)
        elif kind == "empty":
            fn = lambda: L.dg_empty_launch(prm["wgs"])  # noqa: E731
            keep = ()
        else:
            raise ValueError(kind)
        torch.cuda.synchronize()
        L.dg_empty_launch(MARKER_WGS)
        for _ in range(CALLS):
            fn()
        torch.cuda.synchronize()
        recs.append(rec)
        del keep, fn
        torch.cuda.empty_cache()
    L.dg_empty_launch(MARKER_WGS)
    torch.cuda.synchronize()
    os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
    with open(out_path, "w") as fh:
        json.dump({"variants": recs, "calls": CALLS, "marker_wgs": MARKER_WGS}, fh, indent=1,
                  default=lambda o: o.tolist() if hasattr(o, "tolist") else str(o))
    del np
    _log(f"wrote {out_path}")


# ------------------------------------------------------------------ summarise (CPU)

def _read_pmc(d):
    """Dispatches of one rocprofv3 --pmc output folder, in dispatch order:
    [(dispatch_id, kernel_name, grid_size, {counter: value})]."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    disp = {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                did = int(row.get("Dispatch_Id") or row.get("Dispatch_ID"))
                ent = disp.setdefault(did, {"name": row["Kernel_Name"], "grid": int(row["Grid_Size"]),
                                            "c": {}})
                name = row["Counter_Name"]
                ent["c"][name] = ent["c"].get(name, 0.0) + float(row["Counter_Value"])
    return [(k, v["name"], v["grid"], v["c"]) for k, v in sorted(disp.items())]


def _is_marker(name, grid):
    # Grid_Size is reported in work-items (256 per work-group of the empty kernel)
    return "empty_kernel" in name and grid in (MARKER_WGS * 256, MARKER_WGS)


def _ours(name):
    return "dg::" in name or "_ZN2dg" in name


def _windows(dispatches, nvar, calls):
    """Window k: the measured dispatches of variant k, i.e. the unbroken run of
    the library's dispatches right after the k-th marker (the copy probe: its
    first `calls` dispatches).  Set-up work of the next variant (input
    generation, quantised inputs, plan uploads) follows the run."""
    wins, k = [], -1
    i = 0
    while i < len(dispatches):
        did, name, grid, c = dispatches[i]
        if _is_marker(name, grid):
            k += 1
            run = []
            j = i + 1
            while j < len(dispatches) and not _is_marker(dispatches[j][1], dispatches[j][2]):
                if k == 0 and len(run) < calls:          # the copy probe comes first
                    run.append(dispatches[j])
                elif k > 0 and _ours(dispatches[j][1]):
                    run.append(dispatches[j])
                else:
                    break
                j += 1
            wins.append(run)
            i = j
        else:
            i += 1
    if len(wins) < nvar:
        raise ValueError(f"found {len(wins)} marker windows for {nvar} variants")
    return wins[:nvar]


def counted(rec, L):
    """The library's counted features of one variant's call (int64 array), or
    None where there is no count (the copy probe)."""
    k, p = rec["kind"], rec["params"]
    if k == "dg":
        return L.perf_features_count("dg", p["dtype"], p["E"], rec["nunit"], p.get("nmat", 3), rec["tile"],
                                     rec["num_cu"])
    if k == "stencil":
        return L.perf_features_count("stencil", "f32", p["n"])
    if k == "matmul":
        return L.perf_features_count("matmul", "f32", p["n"], num_cu=rec["num_cu"])
    if k == "empty":
        return L.perf_features_count("empty", "f32", p["wgs"])
    if k == "quant":
        return L.perf_features_count("quant", p["to"], p["rows"], p["cols"], 1)
    if k == "adjoint":
        tu, td = rec["tiles_bwd"]
        return (L.perf_features_count("bwd_d", "f32", p["E"], rec["nunit"], 3, td, rec["num_cu"]) +
                L.perf_features_count("bwd_u", "f32", p["E"], rec["nunit"], 3, tu, rec["num_cu"]))
    if k == "batched":
        return L.batched_counts({int(q): i for q, i in rec["plan"].items()}, rec["num_cu"])
    return None


def summarise(variants_path, pmc_dirs, json_out, md_out, command):
    with open(variants_path) as fh:
        V = json.load(fh)
    recs, calls = V["variants"], V["calls"]
    per = {r["id"]: {"kernels": None, "counters": {}} for r in recs}
    for d in pmc_dirs:
        wins = _windows(_read_pmc(d), len(recs), calls)
        for rec, win in zip(recs, wins):
            keep = win
            if len(keep) % calls:
                raise ValueError(f"{rec['id']}: {len(keep)} dispatches for {calls} calls in {d}")
            k = len(keep) // calls
            names = [w[1] for w in keep[-k:]]
            if per[rec["id"]]["kernels"] is None:
                per[rec["id"]]["kernels"] = names
            # the last call's dispatches, summed
            for _, _, _, c in keep[-k:]:
                for name, val in c.items():
                    acc = per[rec["id"]]["counters"]
                    acc[name] = acc.get(name, 0.0) + val
            for _, _, _, c in keep[:k]:
                for name, val in c.items():
                    acc = per[rec["id"]]["counters"]
                    acc.setdefault("first_call", {})
                    acc["first_call"][name] = acc["first_call"].get(name, 0.0) + val
    from paper_1904_09538_amd import _lib as L
    names = L.feature_names()
    out = []
    for r in recs:
        ent = {"id": r["id"], "kind": r["kind"], "params": r["params"], "num_cu": r["num_cu"],
               "tile": r.get("tile"), "nunit": r.get("nunit"), "kernels": per[r["id"]]["kernels"],
               "counters_per_call": {k: v for k, v in per[r["id"]]["counters"].items() if k != "first_call"}}
        if "plan" in r:
            ent["plan"] = {q: {"count": i["count"], "workgroups": i["workgroups"], "tile": i["tile"]}
                           for q, i in r["plan"].items()}
        for extra in ("tiles_bwd",):
            if extra in r:
                ent[extra] = r[extra]
        c = counted(r, L)
        if c is not None:
            ent["features"] = {n: int(v) for n, v in zip(names, c)}
        out.append(ent)
    with open(json_out, "w") as fh:
        json.dump({"calls": calls, "variants": [{k: v for k, v in e.items() if k != "features"} for e in out]},
                  fh, separators=(",", ":"))
    _write_md(out, md_out, command)


def waves_of(rec):
    """Waves the variant's call launches, from its launch shapes (the SQ_WAVES
    counter counts them); None where the shapes are not recorded."""
    k, p = rec["kind"], rec["params"]
    f = rec.get("features")
    if k == "dg" and f:
        return f["workgroups"] * rec["tile"]["waves"]
    if k in ("quant", "adjoint", "stencil", "matmul", "empty") and f:
        return f["workgroups"] * 4        # 256-thread work-groups (quant's set-one launch has 64)
    if k == "batched" and f:
        return f["workgroups"] * 4
    return None


def _write_md(out, md_out, command):
    lines = ["# Hardware counters against counted features", "",
             "Every hot-path kernel at its workload size under `rocprofv3 --pmc`: counters of one call",
             "(the second of two; a call's kernels summed) beside the library's counted features",
             "(`perf_features_count`, equal to the oracle's brute-force walk of the same schedule;",
             "`tests/test_counters.py` checks the counters against both).", "",
             "Commands (five passes, one counter group each, then the summary):", "", "```"] + \
        command.splitlines() + ["```", "",
             "Units.  MFMA flops = (MOPS_F32 + MOPS_F64 + MOPS_BF16 + MOPS_F8) x 512.  LDS bytes =",
             "(SQ_INSTS_LDS_LOAD_BANDWIDTH + SQ_INSTS_LDS_STORE_BANDWIDTH) x 64.  HBM bytes: WRITE_SIZE",
             "x 1 KiB and FETCH_SIZE x 2 KiB, the factors at which the counters read a plain 1 GiB",
             "device copy (row copy_1GiB: FETCH 0.5 GiB, WRITE 1 GiB).  Counted loads exclude the",
             "tags for element tiles re-read by later operator groups (`*_l2`), which the schedule",
             "expects from the XCD's L2.  They do include every lane's read of what the caches serve:",
             "the FP8 element scale each lane of an element reads (same 4 bytes), and the operator",
             "rows each work-group loads (far above the fetch on grids of many rounds).", "",
             "| variant | kernels | waves: counter / launched | MFMA flops: counter / counted | "
             "LDS bytes: counter / counted | HBM written: counter / counted stores | "
             "HBM read: counter / counted loads |", "|---|---|---|---|---|---|---|"]
    for e in out:
        c, f = e["counters_per_call"], e.get("features")
        mf = sum(c.get(k, 0) for k in ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64",
                                        "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F8")) * 512
        lds = (c.get("SQ_INSTS_LDS_LOAD_BANDWIDTH", 0) + c.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0)) * 64
        W, F = c.get("WRITE_SIZE", 0) * 1024, c.get("FETCH_SIZE", 0) * 2048
        kern = ", ".join(sorted({k.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
                                 .replace("dg::", "")[:44] for k in (e["kernels"] or [])}))
        if f:
            fm = f["mfma_f32"] + f["mfma_f64"] + f["mfma_bf16"] + f["mfma_fp8"]
            gl = sum(v for k, v in f.items() if k.startswith("gld_") and not k.endswith("_l2"))
            gs = sum(v for k, v in f.items() if k.startswith("gst_"))
            w = waves_of(e)
            row = (f"{c.get('SQ_WAVES', 0):.0f} / {w if w is not None else '-'}", f"{mf:.6g} / {fm:.6g}",
                   f"{lds:.6g} / {f['lds_bytes']:.6g}",
                   f"{W:.4g} / {gs:.4g} ({W / gs:.3f})" if gs else f"{W:.4g} / 0",
                   f"{F:.4g} / {gl:.4g} ({F / gl:.3f})" if gl else f"{F:.4g} / 0")
        else:
            row = (f"{c.get('SQ_WAVES', 0):.0f}", f"{mf:.6g}", f"{lds:.6g}", f"{W:.4g}", f"{F:.4g}")
        lines.append(f"| {e['id']} | `{kern}` | " + " | ".join(row) + " |")
    lines += ["", "Reading the table.",
              "- MFMA flops agree exactly on every row (the counted flops are those of the executed",
              "  instructions, padding included).",
              "- LDS bytes agree exactly except where an LDS instruction moves less than 64 bytes: the",
              "  counter adds floor(active lanes x size / 64) per instruction.  Those are the batched",
              "  pool's claim (one lane stores the 8-byte tile index: 8 bytes per claim), the",
              "  low-precision kernels' operator-scale staging (8 lanes x 4 bytes per work-group), and",
              "  the ragged last wave-tile of the slab path (dg_f32_p2_100003: scalar LDS accesses of",
              "  3 elements' lanes).",
              "- Wave shuffles (the stencil's halo, the quantiser's row maximum) are LDS instructions",
              "  (SQ_INSTS_LDS) that move no LDS bytes; they are not counted as LDS bytes.",
              "- HBM written equals the counted stores where rows are whole 16-byte vectors (p = 2, 3",
              "  FP32, FP64, stencil, matmul); rows at 4-byte offsets write more (p = 4: 1.33x, fewer",
              "  operator panels per group: 1.61x; p = 5 and the low-precision rows: 1.03-1.08x; the",
              "  batch: 1.11x): partial 32-byte sectors.",
              "- HBM read is below the counted loads where cached data is reused (matmul's operand",
              "  tiles, the pipelined loads' clamped rows) and above them where later operator groups",
              "  miss the L2 for element tiles the schedule expects there (p = 4: 1.52x, p = 5: 2.1x).",
              "- There is no barrier counter on gfx950; barrier counts are pinned by the walk only."]
    with open(md_out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


# ------------------------------------------------------------------ one kernel's profile

def _read_stats(d):
    """Kernel rows of a rocprofv3 --kernel-trace --stats folder:
    {name: (calls, avg_ns, min_ns, max_ns)}."""
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no kernel_stats.csv under {d}")
    out = {}
    with open(files[0], newline="") as fh:
        for row in csv.DictReader(fh):
            out[row["Name"]] = (int(row["Calls"]), float(row["AverageNs"]), float(row["MinNs"]),
                                float(row["MaxNs"]))
    return out


def profile(name, match, trace_dir, fetch_dir, write_dir, commands, md_out, traffic_json, key, sources):
    """Summarise one kernel's rocprofv3 runs: the kernel-trace statistics of
    every kernel, and the kernel's HBM bytes per launch from FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for the plain device
    copy in the same run (bytes / counter KiB).  Writes the markdown summary
    and the traffic entry (with a hash of the kernel's sources, so that a
    changed kernel drops its stale traffic)."""
    import hashlib
    stats = _read_stats(trace_dir)
    fetch = _read_pmc(fetch_dir)
    write = _read_pmc(write_dir)

    def per_launch(disp, counter):
        mine = [c[counter] for _, n, _, c in disp if match in n]
        copy = [(c[counter], g) for _, n, g, c in disp if "copyBuffer" in n]
        if not mine or not copy:
            raise ValueError(f"{counter}: kernel or copy probe missing")
        return sum(mine) / len(mine), copy[-1][0]

    f_kib, f_copy = per_launch(fetch, "FETCH_SIZE")
    w_kib, w_copy = per_launch(write, "WRITE_SIZE")
    copy_bytes = 1 << 30
    fs, ws = copy_bytes / (f_copy * 1024), copy_bytes / (w_copy * 1024)
    rd, wr = f_kib * 1024 * fs, w_kib * 1024 * ws
    h = hashlib.sha256()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for f in sources:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    mine = {n: v for n, v in stats.items() if match in n}
    avg = next(iter(mine.values()))[1] * 1e-9 if mine else None
    lines = [f"# rocprofv3 summary: {name}", "", "## Kernel trace (--kernel-trace --stats)", "", "Command:", "",
             "```", commands[0], "```", "", "| kernel | calls | avg (us) | min (us) | max (us) |", "|---|---|---|---|---|"]
    for n, (calls, a, lo, hi) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1])[:8]:
        lines.append(f"| `{n[:110]}` | {calls} | {a / 1e3:.1f} | {lo / 1e3:.1f} | {hi / 1e3:.1f} |")
    lines += ["", "## HBM traffic (--pmc FETCH_SIZE, then --pmc WRITE_SIZE, separate runs)", "", "Commands:", "",
              "```", commands[1], commands[2], "```", "",
              f"Calibration: a plain 1 GiB device copy (`__amd_rocclr_copyBuffer`) reads FETCH_SIZE = "
              f"{f_copy:.0f} KiB and WRITE_SIZE = {w_copy:.0f} KiB per dispatch,",
              f"so the scale factors are fetch x{fs:.4f} and write x{ws:.4f}.", "",
              "| quantity | per launch |", "|---|---|",
              f"| HBM read (FETCH_SIZE x {fs:.4f}) | {rd:.4e} B |",
              f"| HBM written (WRITE_SIZE x {ws:.4f}) | {wr:.4e} B |",
              f"| total | {rd + wr:.4e} B |"]
    if avg:
        lines.append(f"| average duration (trace) | {avg * 1e6:.1f} us |")
    with open(md_out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    data = {}
    if os.path.exists(traffic_json):
        with open(traffic_json) as fh:
            data = json.load(fh)
    data[key] = {"avg_duration_s": avg, "fetch_scale": fs, "write_scale": ws, "read_bytes": rd,
                 "write_bytes": wr, "hbm_bytes_per_launch": rd + wr, "source_hash": h.hexdigest()[:16],
                 "summary": os.path.relpath(md_out, root)}
    with open(traffic_json, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    return data[key]


def stats_table(trace_dir, title, preamble, command, md_out, top=40):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernels by
    total time)."""
    stats = _read_stats(trace_dir)
    lines = [f"# rocprofv3 summary: {title}", ""] + preamble + ["", "Command:", "", "```", command, "```", "",
                                                                "| kernel | calls | avg (us) | min (us) | max (us) |",
                                                                "|---|---|---|---|---|"]
    for n, (calls, a, lo, hi) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1])[:top]:
        lines.append(f"| `{n[:110]}` | {calls} | {a / 1e3:.1f} | {lo / 1e3:.1f} | {hi / 1e3:.1f} |")
    with open(md_out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--out", required=True)
    s = sub.add_parser("summarise")
    s.add_argument("--variants", required=True)
    s.add_argument("--pmc", nargs="+", required=True)
    s.add_argument("--json", required=True)
    s.add_argument("--md", required=True)
    s.add_argument("--command", default="")
    f = sub.add_parser("profile")
    f.add_argument("--name", required=True)
    f.add_argument("--match", required=True, help="substring of the kernel's name")
    f.add_argument("--trace", required=True)
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--commands", nargs=3, required=True, help="trace, fetch and write commands")
    f.add_argument("--md", required=True)
    f.add_argument("--traffic", required=True)
    f.add_argument("--key", required=True)
    f.add_argument("--sources", nargs="+", required=True)
    t = sub.add_parser("stats")
    t.add_argument("--trace", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--preamble", nargs="*", default=[])
    t.add_argument("--command", required=True)
    t.add_argument("--md", required=True)
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.out)
    elif a.cmd == "stats":
        stats_table(a.trace, a.title, a.preamble, a.command, a.md)
    elif a.cmd == "profile":
        print(json.dumps(profile(a.name, a.match, a.trace, a.fetch, a.write, a.commands, a.md, a.traffic,
                                 a.key, a.sources)))
    else:
        summarise(a.variants, a.pmc, a.json, a.md, a.command)


if __name__ == "__main__":
    main()
