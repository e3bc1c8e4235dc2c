"""Benchmark of the DG differentiation hot path on one MI355X.

Headline (the JSON line's value): DG differentiation FP32, hexahedral p = 3
(nunit = 64, the paper's DG configuration), 3 GLL Kronecker operators, 2^21
elements (the largest point of the calibration suite), u ~ U(-1,1) seed 0.
One step = one dgdiff_apply over all elements, inputs resident in HBM.

The same run measures every other row of the hot path and reports it under
"rows": DG FP32 at p = 2..5; p = 5 at 2^20 elements with BF16 and FP8
operands against FP32; the quantiser; the mixed-order batched launch against
seven plain launches, with the model's predicted time; forward + adjoint at
p = 4; the five-point stencil and matmul companions; and a live calibration
of the performance model (held-out MAPE).

Timing: HIP events on the launch stream over the timed steps.  Before
them every measurement runs its warm-up launches and then keeps launching for
at least WARM_S seconds, whatever --warmup says: after idle the GPU clock
needs about 20 ms of load to settle, and the numbers reported are the steady
rate.  Roofline positions use the algorithmic bytes and flops of one launch
and the MI355X peaks (HBM 8 TB/s, FP32 matrix 157.3 TFLOP/s, BF16 2.5
PFLOP/s, FP8 5.0 PFLOP/s, FP64 78.6 TFLOP/s).

Accuracy: every row keeps the GPU's outputs on a seeded sample of its
elements (the first and last 64 and 2048 drawn at random; the headline keeps
all of them), and the CPU-oracle leg at the end compares them with the FP64
oracle on the same inputs ("err_vs_oracle": normwise max |y - y_ref| /
max |y_ref|).  That leg is the only place this script calls the oracle; it
also times it ("cpu_baseline").
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DG-diff elems/s & %roofline, BF16/FP8/batched vs FP32; perf-model MAPE"
PEAK = {"hbm": 8000.0, "f32": 157.3, "f64": 78.6, "bf16": 2500.0, "fp8": 5000.0}
KERNEL_SOURCES = ["paper_1904_09538_amd/csrc/dg_kernel.hpp",
                  "paper_1904_09538_amd/csrc/dg_forward.hip"]
WARM_S = 0.1          # seconds of launches before any timed region
SAMPLE_RANDOM = 2048  # elements drawn (seed 99) for the accuracy check of a row


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


def kernel_source_hash(files=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(key: str, src_hash: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        ent = json.load(fh).get(key)
    if not ent or ent.get("source_hash") != src_hash:
        return None
    return ent.get("hbm_bytes_per_launch")


def warm(fn, warmup, warm_s=WARM_S):
    """`warmup` calls, then more until at least warm_s seconds have passed: the
    first milliseconds of sustained load after idle run at a transient clock
    (a few launches fast, then a dip, then a slow climb to the steady rate)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def timed(fn, steps, warmup, warm_s=WARM_S):
    """Average seconds per call, HIP events on the current stream, after warm()."""
    import torch
    warm(fn, warmup, warm_s)
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / steps


def roofline(alg_bytes, alg_flops, t, peak_key):
    t_mem = alg_bytes / (PEAK["hbm"] * 1e9)
    t_cmp = alg_flops / (PEAK[peak_key] * 1e12) if alg_flops else 0.0
    if t_cmp >= t_mem:
        r = {"bound": "mfma", "achieved": alg_flops / t / 1e12, "peak": PEAK[peak_key], "unit": "TFLOP/s"}
    else:
        r = {"bound": "hbm", "achieved": alg_bytes / t / 1e9, "peak": PEAK["hbm"], "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    return r


def dg_bytes_flops(E, n, in_bytes, out_bytes, nmat=3):
    return E * n * in_bytes + nmat * E * n * out_bytes + nmat * n * n * in_bytes, 2 * nmat * n * n * E


def sample_elements(E, k=SAMPLE_RANDOM, seed=99):
    """First and last 64 elements and k drawn at random (sorted, unique)."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(min(64, E)), np.arange(max(0, E - 64), E),
                                     rng.integers(0, E, k)])).astype(np.int64)


def gather_out(torch, o, sel):
    """out[:, sel, :] of a [nmat][E][n] device tensor as FP64 [nsel][nmat][n] on the host."""
    idx = torch.from_numpy(sel).to(o.device)
    return o.index_select(1, idx).permute(1, 0, 2).double().cpu().numpy()


# ------------------------------------------------------------------ rows
# Each row returns its measurements and appends accuracy checks to `checks`:
# dicts with the row's place ("at"), the kind of reference and the arrays the
# CPU-oracle leg needs (inputs as FP64 values of what the GPU read, and the
# GPU's outputs on the sample).

def row_dg_orders(L, I, torch, steps, checks):
    out = {}
    for p in (2, 3, 4, 5):
        n, E = (p + 1) ** 3, 1 << 21
        D64 = I.gll_dmats(p).astype(np.float32).astype(np.float64)
        u32 = I.uniform_u(E, n).astype(np.float32)
        D = torch.from_numpy(D64).float().cuda()
        u = torch.from_numpy(u32).cuda()
        o = torch.empty((3, E, n), device="cuda")
        t = timed(lambda: L.dgdiff_apply(D, u, out=o), steps, 2)
        b, f = dg_bytes_flops(E, n, 4, 4)
        key = f"p{p}"
        out[key] = {"nunit": n, "nelem": E, "ms": t * 1e3, "elements_per_s": E / t,
                    "roofline": roofline(b, f, t, "f32")}
        sel = sample_elements(E)
        checks.append({"at": ("dg_fp32_orders_2e21", key), "kind": "dg", "D": D64,
                       "u": u32[sel].astype(np.float64), "got": gather_out(torch, o, sel)})
        log(f"dg fp32 p={p}: {t * 1e3:.3f} ms")
        del D, u, o, u32
        torch.cuda.empty_cache()
    return out


def _codes_to_host(torch, q, sel=None):
    """Raw codes of a BF16 / FP8 tensor (rows `sel` only, if given) as uint16 / uint8."""
    bf = q.dtype == torch.bfloat16
    raw = q.view(torch.int16 if bf else torch.uint8)
    if sel is not None:
        raw = raw.index_select(0, sel)
    h = raw.cpu().numpy()
    return h.view(np.uint16) if bf else h


def row_lowp(L, I, torch, steps, checks):
    p, n, E = 5, 216, 1 << 20
    D64 = I.gll_dmats(p).astype(np.float32).astype(np.float64)
    u32h = I.uniform_u(E, n).astype(np.float32)
    u32 = torch.from_numpy(u32h).cuda()
    Dg = torch.from_numpy(D64).float().cuda()
    o = torch.empty((3, E, n), device="cuda")
    sel = sample_elements(E)
    usel = u32h[sel].astype(np.float64)
    selg = torch.from_numpy(sel).cuda()
    res = {}
    t32 = timed(lambda: L.dgdiff_apply(Dg, u32, out=o), steps, 2)
    b, f = dg_bytes_flops(E, n, 4, 4)
    res["fp32"] = {"ms": t32 * 1e3, "elements_per_s": E / t32, "roofline": roofline(b, f, t32, "f32")}
    checks.append({"at": ("precision_p5_2e20", "fp32"), "kind": "dg", "D": D64, "u": usel,
                   "got": gather_out(torch, o, sel)})
    # default bodies (the staged one at nunit 216), the body with operator
    # panels in LDS for comparison, and the opt-in native FP8 instruction
    for name, to, flags in (("bf16", "bf16", 0), ("fp8", "e4m3", 0), ("bf16_lds_panels", "bf16", 8),
                            ("fp8_lds_panels", "e4m3", 8), ("fp8_native", "e4m3", 2)):
        qD, isD = L.dgdiff_quantize(Dg.reshape(3, -1), to)
        qu, isu = L.dgdiff_quantize(u32, to)
        sc = dict(inv_sD=isD, inv_su=isu) if to == "e4m3" else {}
        tile = dict(flags=flags) if flags else None
        t = timed(lambda: L.dgdiff_apply(qD.view(3, n, n), qu, out=o, tile=tile, **sc), steps, 2)

        # end to end: quantise the element data, then apply (the operator
        # stack is quantised once per operator, outside the loop)
        def e2e():
            q, s = L.dgdiff_quantize(u32, to)
            L.dgdiff_apply(qD.view(3, n, n), q, out=o, tile=tile,
                           **(dict(inv_sD=isD, inv_su=s) if to == "e4m3" else {}))
        te = timed(e2e, steps, 2)
        eb = 2 if to == "bf16" else 1
        b, f = dg_bytes_flops(E, n, eb, 4)
        shape = L.resolve_tile("bf16" if to == "bf16" else "fp8", 3, E, n, tile)
        res[name] = {"body": "lds_panels" if flags else "staged", "shape": shape,
                     "ms": t * 1e3, "elements_per_s": E / t, "speedup_vs_fp32": t32 / t,
                     "quantize_u_and_apply_ms": te * 1e3, "quantize_u_and_apply_speedup_vs_fp32": t32 / te,
                     "roofline": roofline(b, f, t, "bf16" if name != "fp8_native" else "fp8")}
        # the last e2e call wrote o with freshly quantised (identical) codes
        checks.append({"at": ("precision_p5_2e20", name), "kind": "dg_lowp", "fmt": to, "D": D64,
                       "u": usel, "qD": _codes_to_host(torch, qD).reshape(3, n, n),
                       "qu": _codes_to_host(torch, qu, selg),
                       "isD": isD.cpu().numpy().astype(np.float64) if to == "e4m3" else None,
                       "isu": isu.index_select(0, selg).cpu().numpy().astype(np.float64)
                       if to == "e4m3" else None,
                       "got": gather_out(torch, o, sel)})
        log(f"dg {name} p=5 2^20: {t * 1e3:.3f} ms ({t32 / t:.2f}x fp32); "
            f"quantise+apply {te * 1e3:.3f} ms ({t32 / te:.2f}x)")
        del qD, qu, isD, isu
    # BF16 straight from FP32 element data: the staged body rounds u to BF16
    # as it stages it (DG_TILE_QUANT_U), one launch in place of quantise +
    # apply, with the same result bits
    qD, _ = L.dgdiff_quantize(Dg.reshape(3, -1), "bf16")
    fused = dict(flags=L.DG_TILE_QUANT_U)
    tf = timed(lambda: L.dgdiff_apply(qD.view(3, n, n), u32, out=o, tile=fused), steps, 2)
    b, f = dg_bytes_flops(E, n, 4, 4)
    res["bf16_rounded_in_kernel"] = {
        "body": "staged, u FP32 rounded to BF16 while staged", "shape": L.resolve_tile("bf16", 3, E, n, fused),
        "ms": tf * 1e3, "elements_per_s": E / tf, "speedup_vs_fp32": t32 / tf,
        "speedup_vs_quantize_u_and_apply": res["bf16"]["quantize_u_and_apply_ms"] / (tf * 1e3),
        "roofline": roofline(b, f, tf, "bf16")}
    qu, _ = L.dgdiff_quantize(u32, "bf16")
    checks.append({"at": ("precision_p5_2e20", "bf16_rounded_in_kernel"), "kind": "dg_lowp", "fmt": "bf16",
                   "D": D64, "u": usel, "qD": _codes_to_host(torch, qD).reshape(3, n, n),
                   "qu": _codes_to_host(torch, qu, selg), "isD": None, "isu": None,
                   "got": gather_out(torch, o, sel)})
    log(f"dg bf16 rounded in kernel p=5 2^20: {tf * 1e3:.3f} ms ({t32 / tf:.2f}x fp32)")
    del qD, qu
    # the quantiser itself (element data, per-element power-of-two scales)
    tq = timed(lambda: L.dgdiff_quantize(u32, "e4m3"), steps, 2)
    res["quantize_u_fp8"] = {"ms": tq * 1e3, "GB_per_s": (E * n * (4 + 1) + E * 4) / tq / 1e9,
                             "roofline": roofline(E * n * 5 + E * 4, 0, tq, "f32")}
    qu, isu = L.dgdiff_quantize(u32, "e4m3")
    checks.append({"at": ("precision_p5_2e20", "quantize_u_fp8"), "kind": "quant", "x": u32h[sel],
                   "q": _codes_to_host(torch, qu, selg),
                   "inv": isu.index_select(0, selg).cpu().numpy()})
    del u32, o, qu, isu
    torch.cuda.empty_cache()
    return {"config": "hex p=5, 2^20 elements, FP32 output and accumulation", **res}


def row_batched(L, I, torch, steps, model, checks, model_overlap=None):
    E = 1 << 20
    order = I.batched_orders(E)
    off = I.batched_offsets(order)
    total = int(off[-1])
    uh = np.random.default_rng(0).uniform(-1, 1, total).astype(np.float32)
    u = torch.from_numpy(uh).cuda()
    Dh = {p: I.gll_dmats(p).astype(np.float32) for p in range(1, 8)}
    Ds = {p: torch.from_numpy(Dh[p]).cuda() for p in range(1, 8)}
    plan = L.BatchedPlan(order, model=model)
    o = torch.empty((3, total), device="cuda")
    tb = timed(lambda: plan.apply(Ds, u, out=o), steps, 2)
    # the model's predictions of the launch that ran, under the batched-family
    # model: (a) each order priced alone on the whole GPU on the body that
    # runs it (the planner's own estimates, the configuration the family was
    # calibrated on), the orders sharing the GPU so their times add; (b) the
    # counted features of the whole launch (every order's share: work adds,
    # the longest chain is the launch's)
    info = {p: plan.info(p) for p in range(1, 8)}
    pred = sum(i["predicted_s"] for i in info.values() if i["count"]) if model else None
    feats = L.batched_counts(info, torch.cuda.get_device_properties(0).multi_processor_count)
    pred_counts = model_predict(model, feats) if model else None
    mo = model_overlap or (model if model and model.get("group") else None)
    pred_counts_ov = model_predict(mo, feats) if mo else None
    sel = sample_elements(E)
    for p in range(1, 8):
        sp = sel[order[sel] == p]
        if sp.size == 0:
            continue
        n = (p + 1) ** 3
        rows = (off[sp][:, None] + np.arange(n)[None, :]).reshape(-1)
        got = o[:, torch.from_numpy(rows).cuda()].view(3, sp.size, n).permute(1, 0, 2).double().cpu().numpy()
        checks.append({"at": ("batched_mixed_p1_7_2e20", f"order{p}"), "kind": "dg",
                       "D": Dh[p].astype(np.float64), "u": uh[rows].reshape(sp.size, n).astype(np.float64),
                       "got": got})
    # baseline: seven plain launches on pre-grouped copies (grouping not timed)
    groups = {}
    for p in range(1, 8):
        idx = np.nonzero(order == p)[0]
        n = (p + 1) ** 3
        if idx.size == 0:
            continue
        base = torch.from_numpy(off[idx].astype(np.int64)).cuda()
        rows = (base[:, None] + torch.arange(n, device="cuda")[None, :]).reshape(-1)
        ug = u[rows].view(idx.size, n).contiguous()
        groups[p] = (ug, torch.empty((3, idx.size, n), device="cuda"))
        del base, rows

    def seven():
        for p, (ug, og) in groups.items():
            L.dgdiff_apply(Ds[p], ug, out=og)
    t7 = timed(seven, steps, 2)
    flops = sum(2 * 3 * ((p + 1) ** 3) ** 2 * int((order == p).sum()) for p in range(1, 8))
    byts = 4 * 4 * total
    res = {"nelem": E, "total_nodes": total, "ms": tb * 1e3, "elements_per_s": E / tb,
           "roofline": roofline(byts, flops, tb, "f32"),
           "seven_plain_launches_ms": t7 * 1e3, "speedup_vs_plain": t7 / tb,
           "predicted_ms": pred * 1e3 if pred else None,
           "model_rel_error": (pred - tb) / tb if pred else None,
           "predicted_by": "batched-family model: sum of every order's time alone on the GPU, on the body "
                           "that ran it",
           "predicted_ms_launch_counts": pred_counts * 1e3 if pred_counts else None,
           "launch_counts_rel_error": (pred_counts - tb) / tb if pred_counts else None,
           "predicted_ms_launch_counts_overlap_form": pred_counts_ov * 1e3 if pred_counts_ov else None,
           "launch_counts_overlap_form_rel_error": (pred_counts_ov - tb) / tb if pred_counts_ov else None,
           "plan": {p: {k: info[p][k] for k in ("count", "workgroups", "predicted_s")} for p in info},
           "shapes": {p: plan.info(p)["tile"] for p in range(1, 8)}}
    log(f"batched: {tb * 1e3:.3f} ms vs 7 launches {t7 * 1e3:.3f} ms, predicted "
        f"{pred * 1e3 if pred else float('nan'):.3f} ms")
    del u, o, groups
    torch.cuda.empty_cache()
    return res


def row_adjoint(L, I, torch, steps, checks):
    p, n, E = 4, 125, 1 << 19
    D64 = I.gll_dmats(p).astype(np.float32).astype(np.float64)
    u32 = I.uniform_u(E, n).astype(np.float32)
    g32 = I.normal_g(3, E, n).astype(np.float32)
    D = torch.from_numpy(D64).float().cuda()
    u = torch.from_numpy(u32).cuda()
    g = torch.from_numpy(g32).cuda()
    o = torch.empty((3, E, n), device="cuda")
    tf = timed(lambda: L.dgdiff_apply(D, u, out=o), steps, 2)
    tbw = timed(lambda: L.dgdiff_backward(D, u, g), steps, 2)
    gu, gD = L.dgdiff_backward(D, u, g)
    sel = sample_elements(E)
    rng = np.random.default_rng(98)
    ent = (rng.integers(0, 3, 256), rng.integers(0, n, 256), rng.integers(0, n, 256))
    checks.append({"at": ("adjoint_p4_2e19", "forward"), "kind": "dg", "D": D64,
                   "u": u32[sel].astype(np.float64), "got": gather_out(torch, o, sel)})
    checks.append({"at": ("adjoint_p4_2e19", "grad_u"), "kind": "grad_u", "D": D64,
                   "g": g32[:, sel, :].astype(np.float64),
                   "got": gu.index_select(0, torch.from_numpy(sel).cuda()).double().cpu().numpy()})
    checks.append({"at": ("adjoint_p4_2e19", "grad_D"), "kind": "grad_D", "u": u32, "g": g32, "ent": ent,
                   "got": gD.double().cpu().numpy()[ent]})
    flops_f = 2 * 3 * n * n * E
    res = {"config": "hex p=4, 2^19 elements, FP32", "forward_ms": tf * 1e3, "backward_ms": tbw * 1e3,
           "forward_roofline": roofline(E * n * 16, flops_f, tf, "f32"),
           "backward_roofline": roofline(E * n * 4 * 5, 2 * flops_f, tbw, "f32")}
    log(f"adjoint p=4: fwd {tf * 1e3:.3f} ms, bwd {tbw * 1e3:.3f} ms")
    del D, u, g, o, gu, gD
    torch.cuda.empty_cache()
    return res


def row_companions(L, I, torch, steps, checks):
    n = 16384
    grid = I.stencil_grid(n).astype(np.float32)
    ug = torch.zeros((n + 2, n + 64), device="cuda")
    ug[:, :n + 2] = torch.from_numpy(grid).cuda()
    r = torch.empty((n, n), device="cuda")
    ts = timed(lambda: L.stencil5_apply(ug, res=r, n=n), steps, 2)
    st = {"n": n, "ms": ts * 1e3, "points_per_s": n * n / ts,
          "roofline": roofline(((n + 2) ** 2 + n * n) * 4, 5 * n * n, ts, "f32")}
    rng = np.random.default_rng(97)
    ii = np.concatenate([[0, 0, n - 1, n - 1], rng.integers(0, n, 4092)])
    jj = np.concatenate([[0, n - 1, 0, n - 1], rng.integers(0, n, 4092)])
    checks.append({"at": ("stencil5",), "kind": "stencil", "u": grid, "ii": ii, "jj": jj,
                   "got": r[torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()].double().cpu().numpy()})
    del ug, r
    m = 8192
    a, b = I.matmul_operands(m)
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    a = torch.from_numpy(a32).cuda()
    b = torch.from_numpy(b32).cuda()
    c = torch.empty((m, m), device="cuda")
    tm = timed(lambda: L.matmul_apply(a, b, c), max(3, steps // 5), 1)
    mm = {"n": m, "ms": tm * 1e3, "roofline": roofline(12 * m * m, 2 * m ** 3, tm, "f32")}
    ii = np.concatenate([[0, 0, m - 1, m - 1], rng.integers(0, m, 1020)])
    jj = np.concatenate([[0, m - 1, 0, m - 1], rng.integers(0, m, 1020)])
    checks.append({"at": ("matmul",), "kind": "matmul", "a": a32, "b": b32, "ii": ii, "jj": jj,
                   "got": c[torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()].double().cpu().numpy()})
    log(f"stencil n={n}: {ts * 1e3:.3f} ms; matmul n={m}: {tm * 1e3:.3f} ms")
    del a, b, c
    torch.cuda.empty_cache()
    return {"stencil5": st, "matmul": mm}


def achievable_hbm(torch):
    """Measured reference rates of this GPU's memory system: a plain 1 GiB fill
    (write only) and a 1 GiB device-to-device copy (read + write), steady
    state, GB/s."""
    src = torch.ones(1 << 28, device="cuda")
    dst = torch.empty_like(src)
    tf = timed(lambda: dst.fill_(2.0), 20, 2)
    tc = timed(lambda: dst.copy_(src), 20, 2)
    del src, dst
    torch.cuda.empty_cache()
    return {"fill_GBps": (1 << 30) / tf / 1e9, "copy_GBps": 2 * (1 << 30) / tc / 1e9}


def row_model(path):
    import contextlib
    from paper_1904_09538_amd import calibrate as C
    fresh = os.path.splitext(path)[0] + "_fresh.jsonl"
    with contextlib.redirect_stdout(sys.stderr):      # keep stdout to the one JSON line
        C.measure(path, quick=False, trials=60)
        C.measure_fresh(fresh, trials=60)
    s = C.fit_all(path, fresh_path=fresh)
    fams = {k: {"kind": v["kind"], "mape_heldout": v["mape_heldout"],
                "geomean_heldout": v["geomean_heldout"],
                "unconstrained_mape_heldout": v["unconstrained"]["mape_heldout"],
                "unconstrained_negative_params": v["unconstrained"]["negative_params"],
                "n_train": v["n_train"], "n_heldout": v["n_heldout"],
                **({"ranking": v["ranking"]} if "ranking" in v else {})}
            for k, v in s["families"].items()}
    x = s.get("cross")
    cross = None if not x else {
        "trained_on": x["train_families"], "predicts": x["target"], "n_target": x["n_target"],
        "mape": x["nonneg"]["mape"], "geomean": x["nonneg"]["geomean"],
        "ranking": x["nonneg"].get("ranking"), "unconstrained_mape": x["unconstrained"]["mape"]}
    fr = s.get("fresh")
    fresh_row = None if not fr else {
        "seed": fr["seed"], "mape_all": fr["mape_all"], "geomean_all": fr["geomean_all"],
        "families": {k: {"n": v["n"], "mape": v["mape"], "geomean": v["geomean"],
                         **({"ranking": v["ranking"]} if v.get("ranking") else {})}
                     for k, v in fr["families"].items()},
        "protocol": "sizes off the calibration grids, inputs from a fresh seed, scored once by the "
                    "models (forms chosen on the calibration rows) fitted on every calibration row"}
    micro = {t: None if not m else {
        "mape": m["mape"], "geomean": m["geomean"], "linear_mape": m["linear_mape"], "n_target": m["n_target"],
        "n_train": m["n_train"], "trained_on": m["train_kinds"],
        **({"ranking": m["ranking"]} if m.get("ranking") else {})} for t, m in (s.get("micro") or {}).items()}
    ov = s.get("overlap")
    overlap = None if not ov else {
        "overlap_median_per_order": ov["overlap_median_per_order"],
        "reading": "(gmem twin + on-chip from microbenchmark rates - kernel time) / min of the two: "
                   "1 = complete overlap, 0 = none"}
    return s, {"mape_heldout_all": s["mape_heldout_all"],
               "geomean_heldout_all": s["geomean_heldout_all"], "families": fams,
               "cross_kernel": cross, "fresh_heldout": fresh_row,
               "microbenchmark_calibrated": micro, "overlap_diagnosis": overlap,
               "read_pattern_ab": s.get("pattern_ab"),
               "protocol": "cold cache, 60 event-timed trials per variant, 20% held out (seed 4); "
                           "non-negative fit primary, unconstrained fit beside"}


def row_variants(path):
    """The variant-ranking study: the paper's equivalent variants (tiled and
    untiled matmul; DG untiled, u-staged, D-staged, D-staged on transposed
    element data; 16 x 16 and 18 x 18 stencils) predicted by a model fitted
    on measurement kernels only (microbenchmarks, empty launches, the
    variants' work-removed twins), each variant's model form chosen by the
    overlap analysis."""
    import contextlib
    from paper_1904_09538_amd import variant_study as V
    with contextlib.redirect_stdout(sys.stderr):      # keep stdout to the one JSON line
        V.measure(path, trials=20)
    s = V.fit(path)
    return {"per_variant": {v: {k: d[k] for k in ("form", "n", "measured_ms", "predicted_ms", "geomean_rel_err",
                                                    "overlap_index_median")}
                            for v, d in s["per_variant"].items()},
            "ranking": {f: {k: r[k] for k in ("groups", "kendall_tau_mean", "top1_rate", "regret_mean",
                                              "regret_max")} for f, r in s["ranking"].items()},
            "geomean_all": s["geomean_all"], "n_calibration": s["n_calibration"],
            "n_variant_rows": s["n_variant_rows"],
            "protocol": "cold cache, 20 event-timed trials per launch; no variant's time enters the fit"}


def model_vector(summary, names, family="dg", form=None):
    """A family's model of a calibration summary as a per-feature cost vector
    (the non-negative fit, whose costs stay positive wherever the batch's
    orders and sizes fall relative to the calibration set); form="overlap"
    takes the family's overlap-form fit where the chosen form is linear."""
    f = summary["families"][family]
    if form == "overlap" and f["kind"] != "overlap":
        if "overlap_form" not in f:
            return None
        f = {**f, **f["overlap_form"], "kind": "overlap"}
    cost = [0.0] * len(names)
    group = [0] * len(names)
    from paper_1904_09538_amd import calibrate as C
    for feat, p in zip(f["features"], f["params"]):
        cost[names.index(feat)] = p
        group[names.index(feat)] = C.group_of(family, feat)
    if f["kind"] == "linear":
        return {"cost": cost, "group": None}
    return {"cost": cost, "group": group, "edge": f["edge"]}


def model_predict(model, feats):
    """Time of a feature vector under a model_vector (linear or overlap form)."""
    import math
    c = [0.0, 0.0, 0.0]
    for k, (p, f) in enumerate(zip(model["cost"], feats)):
        c[model["group"][k] if model["group"] else 0] += p * float(f)
    if not model["group"]:
        return c[0]
    d = c[1] - c[2]
    return c[0] + c[2] + d * 0.5 * (math.tanh(model["edge"] * d) + 1.0)


# ------------------------------------------------------------------ CPU-oracle leg

def _err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    return num / den if den else num


def oracle_leg(D64, u64, nsample, headline_out, checks, rows):
    """The only use of the FP64 C oracle here: time it on the headline workload
    (single-threaded, the first nsample elements) and compare the headline's
    outputs on those elements and every row's sampled outputs with it."""
    import oracle
    us = np.ascontiguousarray(u64[:nsample])
    t0 = time.perf_counter()
    ref = oracle.dg_forward(D64, us)
    dt = time.perf_counter() - t0
    cpu = {"value": nsample / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
           "sample": f"first {nsample} of the {u64.shape[0]} elements, FP64 single-threaded C "
                     f"oracle, {dt:.1f} s"}
    head_err = _err(headline_out, ref) if headline_out is not None else None
    del ref
    for c in checks:
        k = c["kind"]
        e = {}
        if k == "dg":
            ref = oracle.dg_forward(c["D"], c["u"]).transpose(1, 0, 2)
            e["err_vs_oracle"] = _err(c["got"], ref)
        elif k == "dg_lowp":
            ref = oracle.dg_forward(c["D"], c["u"]).transpose(1, 0, 2)
            e["err_vs_oracle"] = _err(c["got"], ref)     # method: vs the unquantised FP32 inputs
            if c["fmt"] == "bf16":
                Dq = oracle.bf16_decode_array(c["qD"]).astype(np.float64)
                uq = oracle.bf16_decode_array(c["qu"]).astype(np.float64)
            else:
                Dq = oracle.e4m3_decode_array(c["qD"]) * c["isD"][:, None, None]
                uq = oracle.e4m3_decode_array(c["qu"]) * c["isu"][:, None]
            refq = oracle.dg_forward(Dq, uq).transpose(1, 0, 2)
            e["err_vs_oracle_dequantised"] = _err(c["got"], refq)   # kernel alone
        elif k == "quant":
            q, inv = oracle.quantize(c["x"], "e4m3", per_row=True)
            e["codes_equal_oracle"] = bool(np.array_equal(q, c["q"]) and np.array_equal(inv, c["inv"]))
        elif k == "grad_u":
            gu, _ = oracle.dg_adjoint(c["D"], np.zeros((c["g"].shape[1], c["D"].shape[1])), c["g"],
                                      want_u=True, want_D=False)
            e["err_vs_oracle"] = _err(c["got"], gu)
        elif k == "grad_D":
            mm, ii, jj = c["ent"]
            ref = oracle.dg_adjoint_D_select(c["u"], c["g"], mm, ii, jj)
            e["err_vs_oracle_sampled_entries"] = _err(c["got"], ref)
        elif k == "stencil":
            e["err_vs_oracle"] = _err(c["got"], oracle.stencil5_select(c["u"], c["ii"], c["jj"]))
        elif k == "matmul":
            e["err_vs_oracle"] = _err(c["got"], oracle.matmul_select(c["a"], c["b"], c["ii"], c["jj"]))
        node = rows
        for key in c["at"]:
            node = node.setdefault(key, {})
        node.update(e)
        node["oracle_sample"] = ("first/last 64 + 2048 seeded elements" if k in ("dg", "dg_lowp", "grad_u", "quant")
                                 else "256 seeded entries" if k == "grad_D" else "4096/1024 seeded points")
    return cpu, head_err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--rows", default="all",
                    help="comma list of extra rows (orders,lowp,batched,adjoint,companions,model,variants) "
                         "or 'all' or 'none'")
    ap.add_argument("--cpu-baseline", type=int, default=1 << 21,
                    help="elements of the workload the CPU oracle runs on (0: skip the oracle leg)")
    ap.add_argument("--calib-out", default=os.path.join(tempfile.gettempdir(), "dgdiff_bench_calibration.jsonl"),
                    help="where the model row writes its calibration measurements (JSON lines)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 1 GiB device copy three times: its FETCH_SIZE / "
                         "WRITE_SIZE counters calibrate the DG kernel's under rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (a single MI355X); nothing is launched on more than one.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1904_09538_amd import _lib as L, inputs as I

    dev = torch.device("cuda:0")
    if args.copy_probe:
        src = torch.ones(1 << 28, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- headline
    p, E, nmat = 3, 1 << 21, 3
    n = I.nunit_of_order(p)
    log(f"headline: DG FP32 p={p} nunit={n} nelem={E}")
    D64 = I.gll_dmats(p).astype(np.float32).astype(np.float64)
    u32 = I.uniform_u(E, n).astype(np.float32)
    D = torch.from_numpy(D64).float().to(dev)
    u = torch.from_numpy(u32).to(dev)
    out = torch.empty((nmat, E, n), device=dev)
    stream = torch.cuda.current_stream()
    step = lambda: L.dgdiff_apply(D, u, out=out, stream=stream)  # noqa: E731
    warm(step, args.warmup)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t = ev0.elapsed_time(ev1) * 1e-3 / args.steps
    alg_bytes, alg_flops = dg_bytes_flops(E, n, 4, 4)
    roof = roofline(alg_bytes, alg_flops, t, "f32")
    src_hash = kernel_source_hash()
    roof["traffic"] = load_traffic("dg_kernel_f32:dg_fp32_p3_2e21", src_hash)
    roof["kernel"] = "dg_kernel<float,16,1,1,false,true> (paired stores)"
    log(f"headline: {t * 1e3:.3f} ms/step, {E / t:.3e} elements/s")
    nsample = min(args.cpu_baseline, E)
    head_out = out[:, :nsample, :].double().cpu().numpy() if nsample else None
    del D, u, out
    torch.cuda.empty_cache()

    rows, checks = {}, []
    want = ["orders", "lowp", "batched", "adjoint", "companions", "model", "variants"] if args.rows == "all" else \
        ([] if args.rows == "none" else args.rows.split(","))
    small = max(5, args.steps // 5)
    model_summary = None
    if "model" in want:
        os.makedirs(os.path.dirname(os.path.abspath(args.calib_out)), exist_ok=True)
        model_summary, rows["model"] = row_model(args.calib_out)
        log(f"model: held-out MAPE {100 * rows['model']['mape_heldout_all']:.1f}%")
    if "variants" in want:
        rows["variant_ranking"] = row_variants(os.path.splitext(args.calib_out)[0] + "_variants.jsonl")
        log("variants: geo-mean error " + ", ".join(
            f"{v} {100 * d['geomean_rel_err']:.1f}%" for v, d in rows["variant_ranking"]["per_variant"].items()))
    if "orders" in want:
        rows["dg_fp32_orders_2e21"] = row_dg_orders(L, I, torch, small, checks)
    if "lowp" in want:
        rows["precision_p5_2e20"] = row_lowp(L, I, torch, small, checks)
    if "batched" in want:
        have = model_summary and "batched" in model_summary["families"]
        mv = model_vector(model_summary, L.feature_names(), "batched") if have else None
        mo = model_vector(model_summary, L.feature_names(), "batched", form="overlap") if have else None
        rows["batched_mixed_p1_7_2e20"] = row_batched(L, I, torch, small, mv, checks, mo)
    if "adjoint" in want:
        rows["adjoint_p4_2e19"] = row_adjoint(L, I, torch, small, checks)
    if "companions" in want:
        rows.update(row_companions(L, I, torch, small, checks))

    # the roofline against measured achievable rates beside the spec peaks:
    # the FP32 matrix rate the matmul row reaches, the fill and copy rates
    ach = achievable_hbm(torch)
    mm = rows.get("matmul")
    if mm:
        ach["mfma_f32_TFLOPs_matmul"] = mm["roofline"]["achieved"]
        roof["frac_vs_achievable"] = roof["achieved"] / mm["roofline"]["achieved"]
    log(f"achievable: fill {ach['fill_GBps']:.0f} GB/s, copy {ach['copy_GBps']:.0f} GB/s")

    cpu, head_err = None, None
    if nsample:
        log(f"cpu-oracle leg: FP64 oracle on {nsample} headline elements and {len(checks)} row samples")
        cpu, head_err = oracle_leg(D64, u32.astype(np.float64), nsample, head_out, checks, rows)

    rec = {
        "metric": METRIC, "value": E / t, "unit": "elements/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"DG differentiation FP32, hex p={p} (nunit={n}), 3 GLL Kronecker "
                               f"operators, {E} elements, u~U(-1,1) seed 0",
                   "nelem": E, "nunit": n, "nmat": nmat},
        "roofline": roof,
        "err_vs_oracle": head_err,
        "err_vs_oracle_sample": f"first {nsample} elements (normwise, FP64 oracle)" if nsample else None,
        "achievable": ach,
        "cpu_baseline": cpu,
        "rows": rows,
        "wall_s_timed": wall,
        "warm_s": WARM_S,
        "kernel_source_hash": src_hash,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
