"""Calibration of the black-box performance model on this GPU.

Follows the paper's procedure (Sections "Other Features", "Computing Model
Parameters", "Predicting Cost", "Results"): run a set of measurement kernels,
record each one's wall time as the output feature and its counted operation
features as inputs, fit the linear model t ~ sum_k p_k f_k (or the overlap
model) with relative scaling, and predict held-out kernels.  The fit is
unconstrained, as in the paper; a second fit with non-negative weights (the
paper's interpretability criterion) is reported beside it.

Timing protocol (the paper's wall-time feature): warm-up launches, then 60
timed trials for every variant, each bracketed by HIP events on the launch
stream (host-device transfer excluded).  Before each trial a 512 MB scratch
buffer is rewritten on the same stream, so that inputs do not stay resident
in the 256 MB last-level cache ("cold" protocol) and so that the first event
is queued behind GPU work: the pair then measures GPU time, never the host's
launch latency (this matters for the empty kernels, whose run time is a few
microseconds).  Samples above 10x the median are dropped (the paper drops
occasional ~10x anomalies seen on AMD hardware); the model input is the mean
of the kept samples.

Measurement set: the DG forward in FP32 for hexahedral orders p = 1..7
(nunit 8 .. 512) at 2^16..2^21 elements (2^15..2^19 for p = 6, 7) with five
launch shapes each,
the five-point stencil at fourteen n in 1024..16384, square matmul at nineteen
n in 512..8192, and empty kernels with 16..65536 work-groups (launch and
work-group costs).  The paper's model forms are the defaults (linear for the
stencil, overlap for DG and matmul); a family takes the linear form instead
when its cross-validation error on the training rows is lower.
20% of each family's variants are held out (seeded) and scored by MAPE and
by the geometric mean of relative error.

Usage:
  python -m paper_1904_09538_amd.calibrate --measure out.jsonl [--quick]
  python -m paper_1904_09538_amd.calibrate --fit out.jsonl [--json summary.json]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

SEED_SPLIT = 4

# model expressions: the features each family's model uses (the paper builds one
# model per application, with global-memory, on-chip and overhead terms)
# and the cost group of each feature (0 overhead, 1 global memory, 2 on-chip)
GROUP = {"launch": 0, "workgroups": 0, "barrier_x_wg": 0, "wave_tiles": 0, "serial_steps": 0, "lat_steps": 0,
         "gld_dg_u": 1, "gld_dg_u_unal": 1, "gld_dg_u_l2": 1, "gld_dg_d": 1, "gst_dg_out": 1,
         "gst_dg_out_unal": 1,
         "gld_st_u": 1, "gst_st_res": 1, "gld_mm_ab": 1, "gst_mm_c": 1,
         "lds_bytes": 2, "mfma_f64": 2, "mfma_f32": 2, "mfma_bf16": 2, "mfma_fp8": 2,
         "valu_f32": 2, "valu_f64": 2, "gld_ws": 1, "gst_ws": 1, "gld_idx": 1, "gld_ub": 1, "gst_ub": 1,
         "gld_ub_strided": 1, "dg_out_w32": 1, "dg_out_w64": 1,
         "stage_chain": 0}
# the paper's choice: the overlap model for DG and matmul, the linear model for
# the stencil (little overlap observed there); the batched launch and the
# adjoint are contractions like DG (overlap), the quantiser a streaming pass
# like the stencil (linear)
KIND = {"dg": "overlap", "stencil": "linear", "matmul": "overlap", "batched": "overlap",
        "bwd": "overlap", "quant": "overlap"}
# Family-specific cost groups.  The quantiser's wave-steps are round trips
# whose latency overlaps the streaming of other waves' rows (short rows are
# bound by the steps, long ones by the bytes), so they compete with the
# global traffic on the on-chip side of the overlap model.
FAMILY_GROUP = {"quant": {"wave_tiles": 2}}


def group_of(family, feat):
    return FAMILY_GROUP.get(family, {}).get(feat, GROUP[feat])
MODELS = {
    "dg": ["launch", "workgroups", "wave_tiles", "serial_steps", "lat_steps", "gld_dg_u", "gld_dg_u_unal",
           "gld_dg_u_l2",
           "gld_dg_d", "gst_dg_out", "gst_dg_out_unal", "dg_out_w32", "dg_out_w64", "stage_chain", "lds_bytes",
           "mfma_f32"],
    # serial_steps (rows of one strip): small grids are bound by the strip's
    # chain of loads rather than by bandwidth
    "stencil": ["launch", "workgroups", "serial_steps", "gld_st_u", "gst_st_res", "lds_bytes", "valu_f32"],
    "matmul": ["launch", "workgroups", "serial_steps", "barrier_x_wg", "gld_mm_ab", "gst_mm_c",
               "lds_bytes", "mfma_f32"],
    # one order alone in a batched launch, on the body that runs it
    "batched": ["launch", "workgroups", "wave_tiles", "serial_steps", "lat_steps", "stage_chain", "barrier_x_wg",
                "gld_idx",
                "gld_dg_u_unal", "gld_dg_u_l2", "gld_dg_d", "gst_dg_out_unal", "lds_bytes", "mfma_f32",
                "valu_f32"],
    # the adjoint's two steps (grad_u on the GEMM or the contraction kernel;
    # grad_D's split partials and reductions)
    "bwd": ["launch", "workgroups", "serial_steps", "lat_steps", "barrier_x_wg", "gld_dg_u", "gld_dg_u_unal",
            "gld_dg_u_l2", "gld_dg_d", "gld_ws", "gst_ws", "gst_dg_out", "gst_dg_out_unal", "lds_bytes",
            "mfma_f32", "valu_f32"],
    # wave_tiles: wave-steps (four short rows, or one long row, or one trip of
    # the whole-array loops), each a round trip of loads and stores
    "quant": ["launch", "workgroups", "wave_tiles", "serial_steps", "gld_dg_u", "gld_dg_u_unal", "gst_dg_out",
              "gst_dg_out_unal", "gld_ws", "gst_ws", "lds_bytes", "valu_f32"],
}


# ------------------------------------------------------------------ variants

# operator panels per work-group for the reduced-residency shape of each
# order (16 x 4 KQ FP32 panels; 6 of them exceed the 160 KB LDS from p = 6)
_DP_SMALL = {4: 6, 5: 6, 6: 3, 7: 2}


def dg_variants(quick=False):
    out = []
    for p in range(1, 8):
        n = (p + 1) ** 3
        kq = -(-n // 4)
        if p <= 5:
            sizes = [16, 17, 18, 19, 20, 21] if not quick else [16, 18, 20]
        else:
            sizes = [15, 16, 17, 18, 19] if not quick else [15, 17, 19]
        shapes = [dict(), dict(elems_per_wave=16), dict(elems_per_wave=32)]
        if kq <= 32:
            shapes.append(dict(elems_per_wave=64))
        if p >= 4:
            shapes.append(dict(elems_per_wave=16, d_panels=_DP_SMALL[p]))
        else:
            shapes.append(dict(elems_per_wave=32, waves=2))
        for s in sizes:
            for t in shapes:
                out.append({"family": "dg", "p": p, "nunit": n, "nelem": 1 << s, "tile": t})
    return out


def stencil_variants(quick=False):
    ns = ([1024, 1280, 1536, 2048, 2560, 3072, 4096, 5120, 6144, 8192, 10240, 12288, 14336, 16384]
          if not quick else [1024, 4096, 16384])
    return [{"family": "stencil", "n": n} for n in ns]


def matmul_variants(quick=False):
    ns = ([512, 640, 768, 896, 1024, 1280, 1536, 1792, 2048, 2304, 2560, 3072, 3584, 4096, 4608,
           5120, 6144, 7168, 8192] if not quick
          else [512, 2048, 8192])
    return [{"family": "matmul", "n": n} for n in ns]


def empty_variants(quick=False):
    return [{"family": "empty", "wgs": w} for w in (16, 64, 256, 1024, 4096, 16384, 65536)]


def batched_variants(quick=False):
    """One order alone in a batched launch: order 1 on its one-element-per-
    thread body and on resident panels, orders 2..5 on resident panels (two
    column-block counts, and half the operator panels per work-group), orders
    4 and 5 also on GEMM tiles, orders 6 and 7 on GEMM tiles."""
    out = []
    for p in range(1, 8):
        n = (p + 1) ** 3
        sizes = [14, 16, 18, 20] if p <= 5 else [13, 15, 17]
        if quick:
            sizes = sizes[::2]
        if p == 1:
            shapes = [None, {"elems_per_wave": 16}, {"elems_per_wave": 32}]
        elif p <= 5:
            kq = 4 * -(-(-(-n // 4)) // 4)
            max_ppg = (80 * 1024) // (16 * (4 * kq + 4) * 4)
            panels = 3 * -(-n // 16)
            shapes = [{"elems_per_wave": 16}, {"elems_per_wave": 32},
                      {"elems_per_wave": 16, "d_panels": max(1, min(max_ppg, panels) // 2)}]
            if p >= 4:
                shapes.append({"flags": 4})
        else:
            shapes = [None]
        for sz in sizes:
            for t in shapes:
                out.append({"family": "batched", "p": p, "nunit": n, "nelem": 1 << sz, "tile": t})
    return out


def bwd_variants(quick=False):
    """The adjoint's steps alone (grad_u, grad_D), FP32, orders 2..5."""
    out = []
    for p in range(2, 6):
        sizes = [14, 16, 18, 19] if not quick else [14, 18]
        for sz in sizes:
            for step in ("u", "d"):
                out.append({"family": "bwd", "p": p, "nunit": (p + 1) ** 3, "nelem": 1 << sz, "step": step})
    return out


def quant_variants(quick=False):
    """The quantiser: per-row scales (BF16, FP8) over row lengths of the DG
    orders and longer rows; one scale for a whole array (FP8)."""
    out = []
    for to in ("bf16", "fp8"):
        for cols in (27, 64, 125, 216, 512, 2048):
            for sz in ([14, 17, 20] if not quick else [14, 20]):
                if cols * (1 << sz) > (1 << 28):
                    continue
                out.append({"family": "quant", "to": to, "cols": cols, "rows": 1 << sz, "per_row": 1})
    for sz in (14, 17, 20):
        out.append({"family": "quant", "to": "fp8", "cols": 216, "rows": 1 << sz, "per_row": 0})
    return out


def fresh_variants():
    """Variants never measured while the feature sets and model forms were
    chosen: sizes off the calibration grids (3 * 2^k elements, n between
    grid points), inputs from a fresh seed.  Scored once with the models
    fitted on every calibration row."""
    out = []
    for p in (2, 3, 4, 5):
        for t in (dict(), dict(elems_per_wave=16), dict(elems_per_wave=32)):
            out.append({"family": "dg", "p": p, "nunit": (p + 1) ** 3, "nelem": 3 << 18, "tile": t})
    for t in (dict(), dict(elems_per_wave=16)):
        out.append({"family": "dg", "p": 6, "nunit": 343, "nelem": 3 << 16, "tile": t})
    out += [{"family": "stencil", "n": n} for n in (7168, 11264)]
    out += [{"family": "matmul", "n": n} for n in (3328, 5632)]
    for p, t in ((2, {"elems_per_wave": 16}), (2, {"elems_per_wave": 32}), (5, {"elems_per_wave": 16}),
                 (5, {"flags": 4}), (1, None), (6, None)):
        out.append({"family": "batched", "p": p, "nunit": (p + 1) ** 3, "nelem": 3 << 16, "tile": t})
    for p in (3, 4):
        for step in ("u", "d"):
            out.append({"family": "bwd", "p": p, "nunit": (p + 1) ** 3, "nelem": 3 << 16, "step": step})
    for to in ("bf16", "fp8"):
        out.append({"family": "quant", "to": to, "cols": 343, "rows": 3 << 17, "per_row": 1})
    return out


SEED_FRESH = 8


def micro_variants(quick=False):
    """The microbenchmark calibration set (Section "Measurement Kernel Sets for
    Evaluation"): each kernel varies one feature while the others stay fixed.
    Global memory (16-byte streams with 1, 2, 4 inputs; 4-byte loads at
    lane strides 1 and 32), FP32 fused multiply-adds, FP32 and BF16 matrix
    instructions, LDS moves (4 and 16 bytes), barriers, and the local/global
    overlap kernel (one global load, m LDS pairs, one global store)."""
    out = []
    sizes = [16, 18, 20, 22, 24] if not quick else [18, 22]
    for nin in (1, 2, 4):
        for sz in sizes:
            out.append({"family": "micro", "kind": "stream", "n": 1 << sz, "a": nin, "b": 0, "dtype": "f32"})
    for S in (1, 32):
        for sz in (20, 22, 24):
            out.append({"family": "micro", "kind": "strided", "n": 1 << sz, "a": S, "b": 0, "dtype": "f32"})
    for nwg in (1024, 4096):
        for it in (64, 256, 1024):
            out.append({"family": "micro", "kind": "fma", "n": nwg, "a": it, "b": 0, "dtype": "f32"})
            for dt in ("f32", "bf16"):
                out.append({"family": "micro", "kind": "mfma", "n": nwg, "a": it, "b": 0, "dtype": dt})
            for w in (1, 4):
                out.append({"family": "micro", "kind": "lds", "n": nwg, "a": it, "b": w, "dtype": "f32"})
            out.append({"family": "micro", "kind": "barrier", "n": nwg, "a": 4 * it, "b": 0, "dtype": "f32"})
    for m in (0, 1, 2, 4, 6, 8, 12, 16, 24, 32, 48, 64):
        out.append({"family": "micro", "kind": "overlap", "n": 1 << 22, "a": m, "b": 0, "dtype": "f32"})
    # the square matmul's two operand-fetch patterns (a: along rows, b: down
    # rows) over the paper's range of widths
    for n in ((2048, 2560, 3072, 3584) if not quick else (2048, 3584)):
        for pat in (0, 1):
            out.append({"family": "micro", "kind": "tile_read", "n": n, "a": pat, "b": 0, "dtype": "f32"})
    return out


def pattern_costs(rows):
    """Time per load of the tiled read patterns a and b at each width (the
    paper's comparison, Section "Global Memory Access Pattern Features")."""
    t = {}
    for r in rows:
        if r.get("family") == "micro" and r.get("kind") == "tile_read":
            n = r["n"]
            t.setdefault(n, {})[r["a"]] = r["t"]["mean"] / (n * n * (n // 16))
    out = [{"n": n, "a_ns_per_load": 1e9 * v[0], "b_ns_per_load": 1e9 * v[1], "b_over_a": v[1] / v[0]}
           for n, v in sorted(t.items()) if 0 in v and 1 in v]
    return out or None


def twin_variants(quick=False):
    """Work-removed twins (Section "Measurement Workload Synthesis by Work
    Removal Transformation") of the modelled kernels: the DG forward at each
    order with the launch shapes of its calibration set at 2^18 and 2^20
    elements (2^16, 2^18 for orders 6, 7), the stencil and matmul at three
    sizes each."""
    out = []
    for v in dg_variants(quick):
        big = v["p"] >= 6
        if v["nelem"] in ((1 << 16, 1 << 18) if big else (1 << 18, 1 << 20)):
            out.append({**v, "family": "twin", "of": "dg"})
    for n in (2048, 8192, 16384):
        out.append({"family": "twin", "of": "stencil", "n": n})
    for n in (1024, 4096, 8192):
        out.append({"family": "twin", "of": "matmul", "n": n})
    return out


# ------------------------------------------------------------------ timing

def time_launch(fn, trials=60, warmup=5, flush=None):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    samples = []
    for _ in range(trials):
        if flush is not None:
            flush.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        samples.append(e0.elapsed_time(e1) * 1e-3)
    s = np.array(samples)
    med = float(np.median(s))
    kept = s[s <= 10 * med]
    return {"mean": float(kept.mean()), "median": med, "min": float(s.min()),
            "kept": int(kept.size), "dropped": int(s.size - kept.size)}


def measure(path, quick=False, trials=60, families=("dg", "stencil", "matmul", "empty", "batched", "bwd",
                                                    "quant", "micro", "twin")):
    import torch

    from . import _lib, inputs

    dev = torch.device("cuda:0")
    flush = torch.empty(128 << 20, dtype=torch.float32, device=dev)  # 512 MB
    rows = []
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    t_start = time.time()

    def emit(row):
        rows.append(row)
        print(json.dumps({k: row[k] for k in row if k not in ("features",)}), flush=True)

    if "dg" in families:
        cache = {}
        for v in dg_variants(quick):
            n, E = v["nunit"], v["nelem"]
            if n not in cache:
                emax = max(w["nelem"] for w in dg_variants(quick) if w["nunit"] == n)
                D = torch.from_numpy(inputs.gll_dmats(v["p"])).float().to(dev)
                u = torch.from_numpy(inputs.uniform_u(emax, n).astype(np.float32)).to(dev)
                out = torch.empty(3 * emax * n, device=dev)
                cache.clear()
                torch.cuda.empty_cache()
                cache[n] = (D, u, out)
            D, u, out = cache[n]
            uv = u[:E]
            ov = out[:3 * E * n].view(3, E, n)
            try:
                tile = _lib.resolve_tile("f32", 3, E, n, v["tile"])
            except _lib.DGError as err:      # a shape this order cannot take
                print(f"calibrate: skip p={v['p']} nelem={E} tile={v['tile']}: {err}", file=sys.stderr)
                continue
            tm = time_launch(lambda: _lib.dgdiff_apply(D, uv, out=ov, tile=tile), trials, flush=flush)
            feats = _lib.perf_features_count("dg", "f32", E, n, 3, tile, num_cu)
            emit({**v, "tile": tile, "t": tm, "features": feats.tolist()})
        cache.clear()
    if "stencil" in families:
        for v in stencil_variants(quick):
            n = v["n"]
            ld = ((n + 2 + 63) // 64) * 64
            ug = torch.zeros((n + 2, ld), device=dev)
            ug[:, :n + 2] = torch.from_numpy(inputs.stencil_grid(n).astype(np.float32)).to(dev)
            res = torch.empty((n, n), device=dev)
            tm = time_launch(lambda: _lib.stencil5_apply(ug, res=res, n=n), trials, flush=flush)
            emit({**v, "t": tm, "features": _lib.perf_features_count("stencil", "f32", n).tolist()})
            del ug, res
    if "matmul" in families:
        for v in matmul_variants(quick):
            n = v["n"]
            a, b = inputs.matmul_operands(n)
            a = torch.from_numpy(a.astype(np.float32)).to(dev)
            b = torch.from_numpy(b.astype(np.float32)).to(dev)
            c = torch.empty((n, n), device=dev)
            tm = time_launch(lambda: _lib.matmul_apply(a, b, c), trials, flush=flush)
            emit({**v, "t": tm, "features": _lib.perf_features_count("matmul", "f32", n, num_cu=num_cu).tolist()})
            del a, b, c
    if "empty" in families:
        for v in empty_variants(quick):
            # the flush is queued ahead of the first event here too: the event
            # pair then brackets GPU time only, not the host's launch latency
            tm = time_launch(lambda: _lib.dg_empty_launch(v["wgs"]), trials, flush=flush)
            emit({**v, "t": tm, "features": _lib.perf_features_count("empty", "f32", v["wgs"]).tolist()})
    for fam, gen in (("batched", batched_variants), ("bwd", bwd_variants), ("quant", quant_variants),
                     ("micro", micro_variants), ("twin", twin_variants)):
        if fam in families:
            for v in gen(quick):
                r = measure_one(v, trials, flush, num_cu)
                if r is not None:
                    emit(r)
    meta = {"meta": True, "device": torch.cuda.get_device_name(0), "num_cu": num_cu,
            "feature_names": _lib.feature_names(), "trials": trials, "protocol": "cold",
            "seconds": time.time() - t_start}
    with open(path, "w") as fh:
        fh.write(json.dumps(meta) + "\n")
        for r in rows:
            fh.write(json.dumps(r) + "\n")
    return meta, rows


def measure_one(v, trials, flush, num_cu, seed=0):
    """Time one variant of the batched, adjoint or quantiser families (or, for
    the fresh set, any family) and count its features; None if the library
    refuses the shape.  Inputs are drawn on the GPU from `seed` (their values
    do not change the schedule)."""
    import torch

    from . import _lib, inputs

    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    fam = v["family"]
    try:
        if fam == "dg":
            n, E = v["nunit"], v["nelem"]
            D = torch.from_numpy(inputs.gll_dmats(v["p"])).float().to(dev)
            u = torch.rand((E, n), generator=gen, device=dev) * 2 - 1
            out = torch.empty((3, E, n), device=dev)
            tile = _lib.resolve_tile("f32", 3, E, n, v["tile"])
            tm = time_launch(lambda: _lib.dgdiff_apply(D, u, out=out, tile=tile), trials, flush=flush)
            return {**v, "tile": tile, "t": tm,
                    "features": _lib.perf_features_count("dg", "f32", E, n, 3, tile, num_cu).tolist()}
        if fam == "stencil":
            n = v["n"]
            ld = ((n + 2 + 63) // 64) * 64
            ug = torch.rand((n + 2, ld), generator=gen, device=dev)
            res = torch.empty((n, n), device=dev)
            tm = time_launch(lambda: _lib.stencil5_apply(ug, res=res, n=n), trials, flush=flush)
            return {**v, "t": tm, "features": _lib.perf_features_count("stencil", "f32", n).tolist()}
        if fam == "matmul":
            n = v["n"]
            a = torch.randn((n, n), generator=gen, device=dev)
            b = torch.randn((n, n), generator=gen, device=dev)
            c = torch.empty((n, n), device=dev)
            tm = time_launch(lambda: _lib.matmul_apply(a, b, c), trials, flush=flush)
            return {**v, "t": tm,
                    "features": _lib.perf_features_count("matmul", "f32", n, num_cu=num_cu).tolist()}
        if fam == "batched":
            p, E = v["p"], v["nelem"]
            order = np.full(E, p, dtype=np.int8)
            plan = _lib.BatchedPlan(order, tiles={p: v["tile"]} if v["tile"] else None)
            Ds = {p: torch.from_numpy(inputs.gll_dmats(p)).float().to(dev)}
            u = torch.rand(plan.total, generator=gen, device=dev) * 2 - 1
            o = torch.empty((3, plan.total), device=dev)
            tm = time_launch(lambda: plan.apply(Ds, u, out=o), trials, flush=flush)
            info = {p: plan.info(p)}
            return {**v, "shape": info[p]["tile"], "workgroups": info[p]["workgroups"], "t": tm,
                    "features": _lib.batched_counts(info, num_cu).tolist()}
        if fam == "bwd":
            n, E = v["nunit"], v["nelem"]
            D = torch.from_numpy(inputs.gll_dmats(v["p"])).float().to(dev)
            u = torch.rand((E, n), generator=gen, device=dev) * 2 - 1
            g = torch.randn((3, E, n), generator=gen, device=dev)
            want_u = v["step"] == "u"
            tu, td = _lib.resolve_backward("f32", 3, E, n)
            tm = time_launch(lambda: _lib.dgdiff_backward(D, u, g, want_u=want_u, want_D=not want_u), trials,
                             flush=flush)
            f = (_lib.perf_features_count("bwd_u", "f32", E, n, 3, tu, num_cu) if want_u
                 else _lib.perf_features_count("bwd_d", "f32", E, n, 3, td, num_cu))
            return {**v, "shape": tu if want_u else td, "t": tm, "features": f.tolist()}
        if fam == "micro":
            k, n, a_, b_ = v["kind"], v["n"], v["a"], v["b"]
            ins, out = [], None
            if k == "stream":
                ins = [torch.rand(4 * n, generator=gen, device=dev) for _ in range(a_)]
                out = torch.empty(4 * n, device=dev)
            elif k == "strided":
                ins = [torch.rand(n * a_, generator=gen, device=dev)]
                out = torch.empty(n, device=dev)
            elif k in ("fma", "barrier"):
                out = torch.empty(256 * n, device=dev)
            elif k == "mfma":
                out = torch.empty(1024 * n, device=dev)
            elif k == "lds":
                ins = [torch.rand(256 * n * b_, generator=gen, device=dev)]
                out = torch.empty(256 * n * b_, device=dev)
            elif k == "overlap":
                ins = [torch.rand(4 * n, generator=gen, device=dev)]
                out = torch.empty(4 * n, device=dev)
            elif k == "tile_read":
                ins = [torch.rand(n * n, generator=gen, device=dev)]
                out = torch.empty(n * n, device=dev)
            tm = time_launch(lambda: _lib.dg_ubench_run(k, n, ins, out, a=a_, b=b_, dtype=v["dtype"]), trials,
                             flush=flush)
            return {**v, "t": tm,
                    "features": _lib.perf_ubench_count(k, n, a_, b_, v["dtype"], num_cu=num_cu).tolist()}
        if fam == "twin":
            if v["of"] == "dg":
                n, E = v["nunit"], v["nelem"]
                D = torch.rand((3, n, n), generator=gen, device=dev)
                u = torch.rand((E, n), generator=gen, device=dev)
                out = torch.empty((3, E, n), device=dev)
                tile = _lib.resolve_tile("f32", 3, E, n, v["tile"])
                tm = time_launch(lambda: _lib.dg_ubench_run("twin_dg", E, [D, u], out, a=n, b=3, tile=tile),
                                 trials, flush=flush)
                return {**v, "tile": tile, "t": tm,
                        "features": _lib.perf_ubench_count("twin_dg", E, n, 3, tile=tile, num_cu=num_cu).tolist()}
            n = v["n"]
            if v["of"] == "stencil":
                ld = ((n + 2 + 63) // 64) * 64
                ug = torch.rand((n + 2, ld), generator=gen, device=dev)
                res = torch.empty((n, n), device=dev)
                tm = time_launch(lambda: _lib.dg_ubench_run("twin_stencil", n, [ug], res, a=ld, b=n), trials,
                                 flush=flush)
                return {**v, "t": tm, "features": _lib.perf_ubench_count("twin_stencil", n, ld, n).tolist()}
            a = torch.rand((n, n), generator=gen, device=dev)
            b = torch.rand((n, n), generator=gen, device=dev)
            c = torch.empty((n, n), device=dev)
            tm = time_launch(lambda: _lib.dg_ubench_run("twin_matmul", n, [a, b], c), trials, flush=flush)
            return {**v, "t": tm,
                    "features": _lib.perf_ubench_count("twin_matmul", n, num_cu=num_cu).tolist()}
        if fam == "quant":
            x = torch.rand((v["rows"], v["cols"]), generator=gen, device=dev) * 2 - 1
            to = "bf16" if v["to"] == "bf16" else "e4m3"
            tm = time_launch(lambda: _lib.dgdiff_quantize(x, to, per_row=bool(v["per_row"])), trials,
                             flush=flush)
            return {**v, "t": tm, "features": _lib.perf_features_count("quant", v["to"], v["rows"], v["cols"],
                                                                        v["per_row"]).tolist()}
    except _lib.DGError as err:
        print(f"calibrate: skip {v}: {err}", file=sys.stderr)
        return None
    raise ValueError(fam)


def measure_fresh(path, trials=60):
    """Time the fresh held-out set (fresh_variants, inputs from SEED_FRESH)."""
    import torch

    from . import _lib

    dev = torch.device("cuda:0")
    flush = torch.empty(128 << 20, dtype=torch.float32, device=dev)
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    rows = []
    for v in fresh_variants():
        r = measure_one(v, trials, flush, num_cu, seed=SEED_FRESH)
        if r is not None:
            rows.append(r)
            print(json.dumps({k: r[k] for k in r if k != "features"}), flush=True)
        torch.cuda.empty_cache()
    meta = {"meta": True, "fresh": True, "feature_names": _lib.feature_names(), "seed": SEED_FRESH}
    with open(path, "w") as fh:
        fh.write(json.dumps(meta) + "\n")
        for r in rows:
            fh.write(json.dumps(r) + "\n")
    return meta, rows


# ------------------------------------------------------------------ fit

def load(path):
    meta, rows = None, []
    with open(path) as fh:
        for line in fh:
            r = json.loads(line)
            if r.get("meta"):
                meta = r
            else:
                rows.append(r)
    return meta, rows


def split_heldout(n, frac=0.2, seed=SEED_SPLIT):
    rng = np.random.default_rng(seed)
    k = int(math.ceil(frac * n))
    perm = rng.permutation(n)
    return np.sort(perm[k:]), np.sort(perm[:k])


def mape(pred, meas):
    pred, meas = np.asarray(pred), np.asarray(meas)
    return float(np.mean(np.abs(pred - meas) / meas))


def geomean(pred, meas):
    r = np.maximum(np.abs(np.asarray(pred) - np.asarray(meas)) / np.asarray(meas), 1e-6)
    return float(np.exp(np.mean(np.log(r))))


def kendall_tau(a, b):
    """Kendall rank correlation (tau-a) of two equal-length sequences."""
    n = len(a)
    if n < 2:
        return None
    s = 0
    for i in range(n):
        for j in range(i + 1, n):
            s += np.sign(a[i] - a[j]) * np.sign(b[i] - b[j])
    return float(s) / (n * (n - 1) / 2)


def ranking(keys, pred, meas):
    """The paper's main use of a model: ranking equivalent variants.  Rows
    with the same key (one problem, different launch shapes) form a group;
    per group, the Kendall tau between predicted and measured times, whether
    the predicted fastest is the measured fastest, and the slowdown of the
    predicted choice against the measured best (regret)."""
    groups = {}
    for k, p, m in zip(keys, pred, meas):
        groups.setdefault(k, []).append((p, m))
    taus, hits, regrets = [], [], []
    sep_ok = sep_n = 0
    for k, v in groups.items():
        if len(v) < 2:
            continue
        p = [x[0] for x in v]
        m = [x[1] for x in v]
        taus.append(kendall_tau(p, m))
        pick = int(np.argmin(p))
        hits.append(1.0 if m[pick] == min(m) else 0.0)
        regrets.append(m[pick] / min(m) - 1.0)
        # pairs whose measured times differ by at least 10%: ordered right?
        for i in range(len(v)):
            for j in range(i + 1, len(v)):
                if max(m[i], m[j]) >= 1.1 * min(m[i], m[j]):
                    sep_n += 1
                    sep_ok += int((p[i] - p[j]) * (m[i] - m[j]) > 0)
    if not taus:
        return None
    return {"groups": len(taus), "kendall_tau_mean": float(np.mean(taus)),
            "top1_rate": float(np.mean(hits)), "regret_mean": float(np.mean(regrets)),
            "regret_max": float(np.max(regrets)),
            "pairs_apart_10pct": sep_n, "pairs_apart_10pct_ordered": (sep_ok / sep_n) if sep_n else None}


# Starting sharpness of the overlap switch, in units of 1 / median(t): the LM
# fit of the overlap model can stop in a poor local minimum, so it is run from
# each of these and the lowest training residual is kept.
EDGE_STARTS = (1.0, 5.0, 20.0, 100.0, 1000.0)


def fit_overlap(L, F, t, group, p0, nonneg):
    tmed = float(np.median(t))
    best = None
    for q in EDGE_STARTS:
        fit = L.perf_model_fit_overlap(F, t, group, relative=True, p0=p0, edge0=q / tmed, nonneg=nonneg)
        if best is None or fit["resid"] < best["resid"]:
            best = fit
    return best


CV_FOLDS = 5
CV_SEED = 6  # fold assignment of the training rows (seed 4 draws the held-out rows)


def cv_error(L, F, t, extra_F, extra_t, group, kind, folds=CV_FOLDS, seed=CV_SEED):
    """Mean relative error of `kind` (linear or overlap, unconstrained) on the
    training rows F, t by k-fold cross-validation; extra_F, extra_t (the
    empty-kernel rows) are in every fit and never scored."""
    order = np.random.default_rng(seed).permutation(len(t))
    errs = []
    for k in range(folds):
        te = order[k::folds]
        tr = np.setdiff1d(order, te)
        if len(te) == 0 or len(tr) == 0:
            continue
        Fa = np.vstack([F[tr], extra_F]) if extra_F is not None else F[tr]
        ta = np.concatenate([t[tr], extra_t]) if extra_t is not None else t[tr]
        lin = L.perf_model_fit(Fa, ta, relative=True)
        if kind == "linear":
            pred = L.perf_model_predict(F[te], lin["p"])
        else:
            fit = fit_overlap(L, Fa, ta, group, lin["p"], False)
            pred = L.perf_model_predict_overlap(F[te], group, fit["p"], fit["edge"])
        errs.extend(np.abs(pred - t[te]) / t[te])
    return float(np.mean(errs)) if errs else float("inf")


def fit_family(meta, rows, family, L, kind=None, with_overhead_rows=True):
    """Fit one family's model on its training rows (plus the empty-kernel rows,
    which pin the launch and work-group costs) and score the held-out rows.

    The model form is the paper's (overlap for DG and matmul, linear for the
    stencil) unless the linear form has the lower cross-validation error on
    the training rows (the held-out rows take no part in the choice); both
    held-out errors are reported.  The primary fit keeps every cost weight
    >= 0 (the paper's interpretability criterion, Section "Assumptions and
    Limitations": a cost that needs a negative weight is not one); the
    unconstrained fit, as the paper computes it, is reported beside it under
    "unconstrained" with its negative weights listed."""
    names = meta["feature_names"]
    cols = [names.index(f) for f in MODELS[family]]
    group = [group_of(family, f) for f in MODELS[family]]
    fam = [r for r in rows if r["family"] == family]
    F = np.array([[r["features"][c] for c in cols] for r in fam], dtype=np.float64)
    t = np.array([r["t"]["mean"] for r in fam])
    train, held = split_heldout(len(fam))
    Ftr, ttr = F[train], t[train]
    if with_overhead_rows:
        emp = [r for r in rows if r["family"] == "empty"]
        if emp:
            Fe = np.array([[r["features"][c] for c in cols] for r in emp], dtype=np.float64)
            te = np.array([r["t"]["mean"] for r in emp])
            Ftr = np.vstack([Ftr, Fe])
            ttr = np.concatenate([ttr, te])
    cv = None
    if kind is None:
        kind = KIND[family]
        if kind == "overlap":
            ex = len(Ftr) - len(train)
            eF, et = (Ftr[len(train):], ttr[len(train):]) if ex else (None, None)
            cv = {k: cv_error(L, F[train], t[train], eF, et, group, k) for k in ("overlap", "linear")}
            if cv["linear"] < cv["overlap"]:
                kind = "linear"

    def one(nonneg):
        lin = L.perf_model_fit(Ftr, ttr, relative=True, nonneg=nonneg)
        res = {"rank": lin["rank"], "cond": lin["cond"]}
        if kind == "linear":
            p, edge, resid = lin["p"], None, lin["resid"]
            pred = L.perf_model_predict(F, p)
        else:
            fit = fit_overlap(L, Ftr, ttr, group, lin["p"], nonneg)
            p, edge, resid = fit["p"], fit["edge"], fit["resid"]
            res["iters"] = fit["iters"]
            pred = L.perf_model_predict_overlap(F, group, p, edge)
        res["linear_mape_heldout"] = mape(L.perf_model_predict(F, lin["p"])[held], t[held])
        res.update({
            "params": [float(x) for x in p], "edge": edge, "resid": resid,
            "negative_params": [MODELS[family][k] for k in np.nonzero(np.asarray(p) < 0)[0]],
            "mape_train": mape(pred[train], t[train]), "mape_heldout": mape(pred[held], t[held]),
            "geomean_heldout": geomean(pred[held], t[held])})
        return res, pred

    out = {"family": family, "kind": kind, "paper_kind": KIND[family], "cv_error": cv,
           "features": MODELS[family], "groups": group,
           "n_train": int(len(train)), "n_heldout": int(len(held))}
    prim, pred = one(True)
    out.update(prim)
    out["unconstrained"], upred = one(False)
    if family == "batched" and kind == "linear":
        # the overlap form beside the chosen one: a mixed launch runs its
        # orders side by side, memory-bound low orders under MFMA-bound high
        # ones, which a sum of per-order costs cannot express
        chosen, kind = kind, "overlap"
        ov, _ = one(True)
        kind = chosen
        out["overlap_form"] = {k: ov[k] for k in ("params", "edge", "mape_heldout", "negative_params")}
    out["heldout"] = [{"variant": {k: fam[i][k] for k in fam[i] if k not in ("features", "t")},
                       "measured_s": float(t[i]), "predicted_s": float(pred[i])} for i in held]
    if family in ("dg", "batched"):
        # launch shapes of one problem (order, element count), ranked by the
        # model fitted on the training rows
        out["ranking"] = ranking([(r["p"], r["nelem"]) for r in fam], pred, t)
        out["unconstrained"]["ranking"] = ranking([(r["p"], r["nelem"]) for r in fam], upred, t)
    return out


def final_model(meta, rows, family, L, kind):
    """The family's model in the chosen form fitted on every calibration row
    (training and held-out) plus the empty-kernel rows, weights >= 0."""
    names = meta["feature_names"]
    cols = [names.index(f) for f in MODELS[family]]
    group = [group_of(family, f) for f in MODELS[family]]
    use = [r for r in rows if r["family"] in (family, "empty")]
    F = np.array([[r["features"][c] for c in cols] for r in use], dtype=np.float64)
    t = np.array([r["t"]["mean"] for r in use])
    lin = L.perf_model_fit(F, t, relative=True, nonneg=True)
    if kind == "linear":
        return {"kind": kind, "features": MODELS[family], "groups": group,
                "params": [float(x) for x in lin["p"]], "edge": None}
    fit = fit_overlap(L, F, t, group, lin["p"], True)
    return {"kind": kind, "features": MODELS[family], "groups": group,
            "params": [float(x) for x in fit["p"]], "edge": fit["edge"]}


def predict_rows(model, names, rows, L):
    cols = [names.index(f) for f in model["features"]]
    F = np.array([[r["features"][c] for c in cols] for r in rows], dtype=np.float64)
    if model["kind"] == "linear":
        return L.perf_model_predict(F, model["params"])
    return L.perf_model_predict_overlap(F, model["groups"], model["params"], model["edge"])


def score_fresh(summary, cal_path, fresh_path):
    """Score the fresh set once: each family's model, in the form chosen on
    the calibration rows, fitted on all of them, predicts every fresh row.
    MAPE, geomean and (DG, batched) the ranking of the launch shapes."""
    from . import _lib
    meta, rows = load(cal_path)
    fmeta, frows = load(fresh_path)
    if fmeta["feature_names"] != meta["feature_names"]:
        raise ValueError("fresh rows were counted with other feature names")
    out = {"seed": fmeta.get("seed"), "families": {}}
    allp, allm = [], []
    for fam, f in summary["families"].items():
        fr = [r for r in frows if r["family"] == fam]
        if not fr:
            continue
        model = final_model(meta, rows, fam, _lib, f["kind"])
        pred = predict_rows(model, meta["feature_names"], fr, _lib)
        meas = np.array([r["t"]["mean"] for r in fr])
        ent = {"n": len(fr), "kind": model["kind"], "mape": mape(pred, meas), "geomean": geomean(pred, meas),
               "rows": [{"variant": {k: r[k] for k in r if k not in ("features", "t")},
                         "measured_s": float(m), "predicted_s": float(q)} for r, m, q in zip(fr, meas, pred)]}
        if fam in ("dg", "batched"):
            ent["ranking"] = ranking([(r["p"], r["nelem"]) for r in fr], pred, meas)
        out["families"][fam] = ent
        allp += list(pred)
        allm += list(meas)
    out["mape_all"] = mape(allp, allm) if allm else None
    out["geomean_all"] = geomean(allp, allm) if allm else None
    return out


# ------------------------------------------------------------ cross-kernel
# The paper calibrates on kernels other than the one predicted (Section
# "Results": microbenchmarks, then the application kernels).  Here the model
# is fitted on the companion, empty, adjoint and quantiser kernels only and
# predicts the DG forward variants.  Their tagged counts are summed into kernel-independent features
# (global bytes loaded and stored, whatever the array or pattern), so what the
# tags distinguish -- aligned vs unaligned rows, L2 re-reads by other operator
# groups -- is invisible to this model by construction.
GENERIC = {"launch": ("launch",), "workgroups": ("workgroups",), "serial_steps": ("serial_steps",),
           "gld": ("gld_",), "gst": ("gst_",), "lds_bytes": ("lds_bytes",), "mfma_f32": ("mfma_f32",),
           "valu_f32": ("valu_f32",)}
GENERIC_GROUP = {"launch": 0, "workgroups": 0, "serial_steps": 0, "gld": 1, "gst": 1, "lds_bytes": 2,
                 "mfma_f32": 2, "valu_f32": 2}


def generic_features(names, rows):
    """[rows][len(GENERIC)] matrix: each generic feature the sum of the counted
    features whose name equals one of its entries or, for entries ending in
    '_', starts with it."""
    idx = []
    for keys in GENERIC.values():
        idx.append([i for i, nm in enumerate(names)
                    if any(nm == k or (k.endswith("_") and nm.startswith(k)) for k in keys)])
    return np.array([[sum(r["features"][i] for i in ix) for ix in idx] for r in rows], dtype=np.float64)


def fit_cross(meta, rows, L, train=("stencil", "matmul", "empty", "bwd", "quant"), target="dg"):
    """Overlap model on the generic features, fitted on the `train` families,
    scored on every `target` row (non-negative fit, and the unconstrained one
    beside it)."""
    names = meta["feature_names"]
    tr = [r for r in rows if r["family"] in train]
    tg = [r for r in rows if r["family"] == target]
    if not tr or not tg:
        return None
    Ftr, ttr = generic_features(names, tr), np.array([r["t"]["mean"] for r in tr])
    Ftg, ttg = generic_features(names, tg), np.array([r["t"]["mean"] for r in tg])
    group = [GENERIC_GROUP[k] for k in GENERIC]
    out = {"train_families": list(train), "target": target, "features": list(GENERIC),
           "n_train": len(tr), "n_target": len(tg)}
    for label, nonneg in (("nonneg", True), ("unconstrained", False)):
        lin = L.perf_model_fit(Ftr, ttr, relative=True, nonneg=nonneg)
        fit = fit_overlap(L, Ftr, ttr, group, lin["p"], nonneg)
        pred = L.perf_model_predict_overlap(Ftg, group, fit["p"], fit["edge"])
        res = {"mape": mape(pred, ttg), "geomean": geomean(pred, ttg),
               "mape_train": mape(L.perf_model_predict_overlap(Ftr, group, fit["p"], fit["edge"]), ttr),
               "params": [float(x) for x in fit["p"]], "edge": fit["edge"]}
        if target == "dg":
            res["ranking"] = ranking([(r["p"], r["nelem"]) for r in tg], pred, ttg)
        out[label] = res
    return out


# ------------------------------------------------------ microbenchmark calibration
# The paper's protocol (Section "Measurement Kernel Sets for Evaluation"):
# the model of a computation is calibrated on measurement kernels that do not
# include it -- microbenchmarks, each exercising one feature, and the
# work-removed twins of the computation, which measure its global-memory
# access pattern alone -- and then predicts the computation.
MICRO_EXTRA = ["gld_ub", "gst_ub", "gld_ub_strided", "valu_f32", "barrier_x_wg", "lds_bytes", "mfma_f32",
               "mfma_bf16"]


def micro_features(target):
    """The target's own model features, plus the microbenchmarks' global-
    memory, VALU and matrix features (zero for the target; they carry the
    microbenchmarks' own costs)."""
    return list(dict.fromkeys(MODELS[target] + MICRO_EXTRA))


def fit_micro(meta, rows, L, target):
    """Overlap model (weights >= 0) of `target` fitted on the microbenchmarks,
    the target's twins and the empty kernels only; scored on every target
    row.  The linear model on the same rows is reported beside it."""
    names = meta["feature_names"]
    feats = micro_features(target)
    cols = [names.index(f) for f in feats]
    group = [GROUP[f] for f in feats]
    tr = [r for r in rows if r["family"] in ("micro", "empty") or
          (r["family"] == "twin" and r.get("of") == target)]
    tg = [r for r in rows if r["family"] == target]
    if not tg or not any(r["family"] == "micro" for r in tr):
        return None
    Ftr = np.array([[r["features"][c] for c in cols] for r in tr], dtype=np.float64)
    ttr = np.array([r["t"]["mean"] for r in tr])
    Ftg = np.array([[r["features"][c] for c in cols] for r in tg], dtype=np.float64)
    ttg = np.array([r["t"]["mean"] for r in tg])
    lin = L.perf_model_fit(Ftr, ttr, relative=True, nonneg=True)
    fit = fit_overlap(L, Ftr, ttr, group, lin["p"], True)
    pred = L.perf_model_predict_overlap(Ftg, group, fit["p"], fit["edge"])
    lpred = L.perf_model_predict(Ftg, lin["p"])
    out = {"target": target, "features": feats, "groups": group, "n_train": len(tr), "n_target": len(tg),
           "train_kinds": sorted({r.get("kind", r["family"]) if r["family"] == "micro" else
                                  ("twin" if r["family"] == "twin" else r["family"]) for r in tr}),
           "params": [float(x) for x in fit["p"]], "edge": fit["edge"],
           "mape_train": mape(L.perf_model_predict_overlap(Ftr, group, fit["p"], fit["edge"]), ttr),
           "mape": mape(pred, ttg), "geomean": geomean(pred, ttg),
           "linear_mape": mape(lpred, ttg)}
    if target == "dg":
        out["ranking"] = ranking([(r["p"], r["nelem"]) for r in tg], pred, ttg)
    return out


def overlap_diagnosis(meta, rows, micro_fit):
    """The paper's use of the work remover to decide on an overlap model: for
    each DG problem with a twin measured at the same launch shape, the twin's
    time (global memory alone), the on-chip time the microbenchmark rates
    give for the kernel's LDS and matrix work, and the kernel's time.  A
    kernel time near max(gmem, on-chip) means the two overlap; near their
    sum, they do not.  overlap = (gmem + on_chip - t) / min(gmem, on_chip):
    1 for complete overlap, 0 for none."""
    if not micro_fit:
        return None
    names = meta["feature_names"]
    p = dict(zip(micro_fit["features"], micro_fit["params"]))
    onchip_feats = [f for f, g in zip(micro_fit["features"], micro_fit["groups"]) if g == 2]
    key = lambda r: (r["p"], r["nelem"], json.dumps(r["tile"], sort_keys=True))  # noqa: E731
    twins = {key(r): r for r in rows if r["family"] == "twin" and r.get("of") == "dg"}
    out = []
    for r in rows:
        if r["family"] != "dg" or key(r) not in twins:
            continue
        f = dict(zip(names, r["features"]))
        onchip = sum(p[k] * f[k] for k in onchip_feats)
        gmem = twins[key(r)]["t"]["mean"]
        t = r["t"]["mean"]
        lo = min(gmem, onchip)
        out.append({"p": r["p"], "nelem": r["nelem"], "tile": r["tile"], "t": t, "gmem_twin": gmem,
                    "onchip_micro": onchip, "overlap": (gmem + onchip - t) / lo if lo > 0 else None})
    if not out:
        return None
    per_order = {}
    for d in out:
        per_order.setdefault(d["p"], []).append(d["overlap"])
    return {"rows": out, "overlap_median_per_order": {k: float(np.median([x for x in v if x is not None]))
                                                      for k, v in sorted(per_order.items())}}


def fit_all(path, kinds=None, fresh_path=None):
    from . import _lib
    meta, rows = load(path)
    out = {"device": meta["device"], "protocol": meta["protocol"], "families": {}}
    for fam in MODELS:
        if any(r["family"] == fam for r in rows):
            out["families"][fam] = fit_family(meta, rows, fam, _lib, (kinds or {}).get(fam))
    allp, allm = [], []
    for f in out["families"].values():
        allp += [h["predicted_s"] for h in f["heldout"]]
        allm += [h["measured_s"] for h in f["heldout"]]
    out["mape_heldout_all"] = mape(allp, allm) if allm else None
    out["geomean_heldout_all"] = geomean(allp, allm) if allm else None
    out["cross"] = fit_cross(meta, rows, _lib)
    out["micro"] = {t: fit_micro(meta, rows, _lib, t) for t in ("dg", "stencil", "matmul")}
    out["overlap"] = overlap_diagnosis(meta, rows, out["micro"]["dg"])
    if fresh_path:
        out["fresh"] = score_fresh(out, path, fresh_path)
    out["pattern_ab"] = pattern_costs(rows)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--measure")
    ap.add_argument("--fit")
    ap.add_argument("--json")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--trials", type=int, default=60)
    ap.add_argument("--families", default="dg,stencil,matmul,empty,batched,bwd,quant,micro,twin")
    ap.add_argument("--fresh", help="measure the fresh held-out set into this file (with --measure), "
                                    "or score it (with --fit)")
    a = ap.parse_args(argv)
    if a.measure:
        measure(a.measure, quick=a.quick, trials=a.trials, families=tuple(a.families.split(",")))
        if a.fresh:
            measure_fresh(a.fresh, trials=a.trials)
    if a.fit:
        s = fit_all(a.fit, fresh_path=a.fresh)
        for fam, f in s["families"].items():
            extra = (f"  (linear model: {100 * f['linear_mape_heldout']:.1f}%)"
                     if "linear_mape_heldout" in f else "")
            print(f"{fam} [{f['kind']}]: held-out MAPE {100 * f['mape_heldout']:.1f}%  geomean "
                  f"{100 * f['geomean_heldout']:.1f}%  train MAPE {100 * f['mape_train']:.1f}%  "
                  f"rank {f['rank']}/{len(f['features'])}  negative {f['negative_params']}{extra}")
        print(f"all families: held-out MAPE {100 * s['mape_heldout_all']:.1f}%")
        if "fresh" in s:
            print(f"fresh set (seed {s['fresh']['seed']}): MAPE {100 * s['fresh']['mape_all']:.1f}%")
        for t, m in (s.get("micro") or {}).items():
            if m:
                print(f"microbenchmark-calibrated {t}: MAPE {100 * m['mape']:.1f}% (linear {100 * m['linear_mape']:.1f}%)")
        if a.json:
            with open(a.json, "w") as fh:
                json.dump(s, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
