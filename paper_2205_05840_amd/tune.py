"""Autotuner of the library's launch shapes, run on the device.

Sweeps, per mesh size, precision, operator mode and class of pairs per launch:
* the plane-marching operator kernel: every launch variant (waves per workgroup, ring
  depth) and a ladder of planes per workgroup, each timed over rotating vector sets larger
  than the last-level cache (ndmg_time_stencil);
* the vertex patch products: 16-vertex groups per wave for the interior segment and for
  the segments on the box's faces and edges, each timed on a fresh context (the shape
  decides the chunk table at setup) over repeated launches of the kernel alone
  (ndmg_level_op with NDMG_OP_PATCH).
The fastest shape of each sweep, with the cost model's choice timed beside it, goes into a
table keyed to the kernel sources (ndmg_source_key), which the binding loads with the
library.  No entry is written where the model's choice is within 2 % of the best.

    python -m paper_2205_05840_amd.tune [--out FILE] [--report FILE] [--quick]
"""
import argparse
import ctypes
import json
import os
import sys

from . import _lib

PREC = {"fp64": 0, "fp32": 1}
KZ_LADDER = (2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128)
# an entry is written only where the measured best beats the cost model's choice by this
# fraction (smaller differences are within the run-to-run spread of the timings)
MIN_GAIN = 0.02


def _stencil_cases(quick):
    sizes = (64, 96, 128) if quick else (40, 48, 56, 64, 80, 96, 112, 128)
    for n in sizes:
        for prec, modes in (("fp64", (0, 1, 2)), ("fp32", (0, 1))):
            for mode in modes:
                yield n, prec, mode, 1
    if not quick:
        # batched classes of the uneven-size form (the operator kernel from n > 16 at >= 4
        # pairs)
        for n in (24, 32):
            for mode in (0, 1, 2):
                yield n, "fp64", mode, 400
            for mode in (0, 1):
                yield n, "fp32", mode, 400


def _time_stencil(torch, n, prec, mode, count, variant, kz, bufs):
    L = _lib.lib()
    x, b, y, part, alpha, nrot = bufs
    out = ctypes.c_double()
    code = L.ndmg_time_stencil(n, PREC[prec], mode, count, variant, kz, x.data_ptr(), b.data_ptr(),
                               y.data_ptr(), part.data_ptr(), alpha.data_ptr(), 20, nrot,
                               torch.cuda.current_stream().cuda_stream, ctypes.byref(out))
    if code == _lib.NDMG_EINVAL:
        return None
    _lib.check(code)
    return out.value


def _stencil_buffers(torch, n, prec, count):
    P = ((n + 1) + 7) // 8 * 8
    vlen = 3 * (n + 1) ** 2 * P
    dt = torch.float64 if prec == "fp64" else torch.float32
    nbytes = count * vlen * (8 if prec == "fp64" else 4)
    nrot = max(1, min(8, -(-512 * 2 ** 20 // (2 * nbytes))))   # rotate over >= 512 MB of x and y
    x = torch.randn(nrot * count * vlen, dtype=dt, device="cuda")
    b = torch.randn(nrot * count * vlen, dtype=dt, device="cuda")
    y = torch.zeros(nrot * count * vlen, dtype=dt, device="cuda")
    part = torch.zeros(count * (n * n + 64), dtype=torch.float64, device="cuda")
    alpha = torch.ones(count, dtype=torch.float64, device="cuda")
    return x, b, y, part, alpha, nrot


def _model_shape(n, prec, mode, count):
    v, z = ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.lib().ndmg_stencil_shape(n, PREC[prec], mode, count, ctypes.byref(v), ctypes.byref(z)))
    return v.value, z.value


def tune_stencil(torch, quick, log):
    entries, report = [], []
    for n, prec, mode, count in _stencil_cases(quick):
        bufs = _stencil_buffers(torch, n, prec, count)
        model = _model_shape(n, prec, mode, count)
        times = {}
        ladder = sorted(set(k for k in KZ_LADDER + (n, model[1]) if 2 <= k <= n))
        for variant in range(8):   # the library refuses a variant past its last
            t = _time_stencil(torch, n, prec, mode, count, variant, ladder[0], bufs)
            if t is None:
                break
            times[(variant, ladder[0])] = t
            for kz in ladder[1:]:
                times[(variant, kz)] = _time_stencil(torch, n, prec, mode, count, variant, kz, bufs)
        best = min(times, key=times.get)
        t_model = times.get(model) or _time_stencil(torch, n, prec, mode, count, model[0], model[1], bufs)
        cls = _class(count)
        rec = {"kernel": "stencil", "n": n, "precision": prec, "mode": mode, "pairs": count,
               "model": list(model), "model_us": t_model, "best": list(best), "best_us": times[best]}
        report.append(rec)
        log(f"stencil n={n} {prec} mode {mode} pairs {count}: model {model} {t_model:.2f} us, "
            f"best {best} {times[best]:.2f} us")
        if times[best] < (1.0 - MIN_GAIN) * t_model:
            entries.append(f"stencil {n} {prec} {mode} {cls} {best[0]} {best[1]}")
        del bufs
        torch.cuda.empty_cache()
    return entries, report


def _class(count):
    return 0 if count <= 1 else 1 if count <= 3 else 2 if count <= 15 else 3 if count <= 63 else 4


def _time_patch(torch, Solver, n, prec, reps=30):
    S = Solver(n, 1.0, precision=prec)
    r = (torch.randn(S.vec_len, dtype=torch.float64, device=S.device) * S.unknown_mask()).contiguous()
    S.level_op(-1, "smooth", r)
    L = _lib.lib()
    ptr = r.data_ptr()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        _lib.check(L.ndmg_level_op(S.ctx, -1, _lib.NDMG_OP_PATCH, ptr, ptr))
    e0.record(S.stream)
    for _ in range(reps):
        _lib.check(L.ndmg_level_op(S.ctx, -1, _lib.NDMG_OP_PATCH, ptr, ptr))
    e1.record(S.stream)
    e1.synchronize()
    S.close()
    return e0.elapsed_time(e1) * 1e3 / reps


def tune_patch(torch, quick, log, keep):
    from .solver import Solver
    L = _lib.lib()
    entries, report = [], []
    sizes = (64, 128) if quick else (48, 64, 96, 128)
    for n in sizes:
        for prec in ("fp32", "fp64"):
            # the table as kept so far (the operator shapes), without a patch entry here
            L.ndmg_tuning_clear()
            for e in keep:
                _lib.check(L.ndmg_tuning_set(e.encode()))
            t_model = _time_patch(torch, Solver, n, prec)
            times = {}
            for gi in range(1, 9):
                for gb in (1, 2, 4):
                    if gb > gi:
                        continue
                    line = f"patch {n} {prec} 0 0 {gi} {gb}"
                    _lib.check(L.ndmg_tuning_set(line.encode()))
                    times[(gi, gb)] = _time_patch(torch, Solver, n, prec)
            best = min(times, key=times.get)
            rec = {"kernel": "patch", "n": n, "precision": prec, "model_us": t_model, "best": list(best),
                   "best_us": times[best]}
            report.append(rec)
            log(f"patch n={n} {prec}: model {t_model:.2f} us, best {best} {times[best]:.2f} us")
            if times[best] < (1.0 - MIN_GAIN) * t_model:
                entries.append(f"patch {n} {prec} 0 0 {best[0]} {best[1]}")
    return entries, report


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=_lib.TUNING_PATH)
    ap.add_argument("--report", default=None, help="JSON lines of every sweep (model and best)")
    ap.add_argument("--quick", action="store_true", help="a few sizes only")
    args = ap.parse_args(argv)
    import torch
    L = _lib.lib()
    L.ndmg_tuning_clear()   # measure the cost model's own choices

    def log(msg):
        print(f"[tune] {msg}", file=sys.stderr, flush=True)

    st_entries, st_report = tune_stencil(torch, args.quick, log)
    pa_entries, pa_report = tune_patch(torch, args.quick, log, st_entries)
    key = L.ndmg_source_key().decode()
    tmp = args.out + ".tmp"
    with open(tmp, "w") as f:
        f.write("# launch shapes measured by paper_2205_05840_amd/tune.py on the device; valid for the\n")
        f.write("# kernel sources of the key below only (the library refuses the table otherwise)\n")
        f.write(f"key {key}\n")
        for e in st_entries + pa_entries:
            f.write(e + "\n")
    os.replace(tmp, args.out)
    if args.report:
        with open(args.report, "w") as f:
            for rec in st_report + pa_report:
                f.write(json.dumps(rec) + "\n")
    _lib.check(L.ndmg_tuning_load(args.out.encode()))
    log(f"wrote {len(st_entries) + len(pa_entries)} entries to {args.out} (key {key})")


if __name__ == "__main__":
    main()
