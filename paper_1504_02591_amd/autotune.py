"""Autotuner for the transform tile shapes and the middle radix split (csrc/recon_tuning.h).

Knobs (compile-time, see recon_tuning.h): RECON_TILE_Z (packed z column pairs per block),
RECON_TILE_Y (y-pass columns), RECON_TILE_X (x-pass rows), RECON_MID_512 / RECON_MID_1024
(split of the middle radix factor), RECON_Z_TPB (z tiles per block of the z iteration, whose
next tile is staged while the current one is finished), RECON_Z_WAVE (wave-local z iteration at
512^3), and per-size copies of the tile and tiles-per-block knobs for 256^3 (_256) and 1024^3
(_1024).  Each grid size tunes its own knobs (SIZE_KNOBS), one knob at a time around the current
setting: every single-knob variant is compiled (in parallel, on the host), each is timed on the GPU
in a process of its own on the correction pass of an n^3 field, or of a batch of them (the dominant
cost of a reconstruction), and each knob takes its fastest value.  The combined choice is timed
again against the current setting and written to recon_tuning.h only if it is faster; the other
sizes' knobs and timings are kept.

    python -m paper_1504_02591_amd.autotune build --dir DIR --n 256 --batch 64   # host: compile
    python -m paper_1504_02591_amd.autotune time --dir DIR                       # GPU: time, pick
    python -m paper_1504_02591_amd.autotune combined --dir DIR                   # build + time the pick
    python -m paper_1504_02591_amd.autotune write --dir DIR                      # host: write the header
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import re
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TUNING = os.path.join(HERE, "csrc", "recon_tuning.h")
# knobs timed at each grid size (recon_tuning.h): the general ones at 512^3 (every size without its own
# values takes them), the per-size ones at 256^3 (the batched workload) and 1024^3
SIZE_KNOBS = {
    512: {"RECON_TILE_Z": [8, 16], "RECON_TILE_Y": [8, 16], "RECON_TILE_X": [2, 4, 8], "RECON_MID_512": [0, 1, 2],
          "RECON_Z_TPB": [1, 2, 4, 8], "RECON_Z_WAVE": [0, 1]},
    256: {"RECON_TILE_Z_256": [8, 16], "RECON_TILE_Y_256": [8, 16], "RECON_TILE_X_256": [2, 4, 8],
          "RECON_Z_TPB_256": [1, 2, 4, 8]},
    1024: {"RECON_TILE_X_1024": [2, 4, 8], "RECON_MID_1024": [0, 1, 2], "RECON_Z_TPB_1024": [1, 2, 4, 8]},
}
KNOBS = {k: v for d in SIZE_KNOBS.values() for k, v in d.items()}


def current():
    """Knob values in recon_tuning.h (a per-size knob defined as a general one takes its value)."""
    text = open(TUNING).read()
    raw = dict(re.findall(r"#define\s+(RECON_\w+)\s+(\w+)", text))
    vals = {}
    for k in KNOBS:
        v = raw[k]
        vals[k] = int(raw[v]) if v in raw else int(v)
    return vals


def variants(base, n):
    """The current setting plus every single-knob deviation of the knobs tuned at grid n."""
    out = {"base": dict(base)}
    for k, choices in SIZE_KNOBS[n].items():
        for v in choices:
            if v != base[k]:
                cfg = dict(base)
                cfg[k] = v
                out[f"{k}={v}"] = cfg
    return out


def _build_one(args):
    name, cfg, out = args
    from paper_1504_02591_amd import build
    flags = [f"-D{k}={v}" for k, v in cfg.items()]
    t0 = time.time()
    build.build(output=out, extra=flags)
    return name, time.time() - t0


def cmd_build(a):
    os.makedirs(a.dir, exist_ok=True)
    base = current()
    vs = variants(base, a.n)
    jobs = [(name, cfg, os.path.join(a.dir, f"lib_{i}.so")) for i, (name, cfg) in enumerate(vs.items())]
    with cf.ProcessPoolExecutor(max_workers=a.jobs) as ex:
        for name, dt in ex.map(_build_one, jobs):
            print(f"[autotune] built {name} in {dt:.0f}s", flush=True)
    meta = {"n": a.n, "batch": a.batch, "base": base,
            "variants": {name: {"cfg": cfg, "lib": os.path.basename(lib)} for name, cfg, lib in jobs}}
    json.dump(meta, open(os.path.join(a.dir, "variants.json"), "w"), indent=1)


def cmd_one(a):
    """Time the correction pass of one library variant (run in a fresh process)."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_1504_02591_amd import native
    native._LIB = native.load(a.lib)
    torch.cuda.set_device(0)
    from synth import generators as G
    n, box = a.n, 3500.0 * a.n / 512
    cache = os.path.join(a.field_cache, f"autotune_field_{n}.npy") if a.field_cache else None
    if cache and os.path.exists(cache):
        field = np.load(cache, allow_pickle=False)
    else:
        field, _ = G.linear_field(n, box, 5, want_psi=False, dtype=np.float32 if n > 512 else np.float64)
        field = np.ascontiguousarray(field, dtype=np.float32)
        if cache:
            np.save(cache, field)
    delta = torch.from_numpy(field).cuda()
    if a.batch > 1:
        delta = delta.unsqueeze(0).expand(a.batch, n, n, n).contiguous()
    # observer outside the box: the iteration contracts for any field, so fixed passes never diverge
    plan = native.Plan(n, box, (box / 2, box / 2, -3.0 * box), 2.0, 0.74, 15.0, randoms=False, batch=a.batch)
    plan.set_delta(delta)
    plan.solve()
    plan.iterate(2, 0.0)
    best = None
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.iterate(a.passes, 0.0)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / a.passes
        best = ms if best is None else min(best, ms)
    plan.close()
    print(json.dumps({"ms_per_pass": best}), flush=True)


def _time(lib, n, passes, batch=1):
    # the variants of one size share the synthetic field, drawn once into the host's temporary directory
    cache = os.environ.get("TMPDIR", "/tmp")
    r = subprocess.run([sys.executable, "-m", "paper_1504_02591_amd.autotune", "one", "--lib", lib, "--n", str(n),
                        "--passes", str(passes), "--batch", str(batch), "--field-cache", cache], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        raise RuntimeError(f"timing {lib} failed:\n{r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])["ms_per_pass"]


def cmd_time(a):
    meta = json.load(open(os.path.join(a.dir, "variants.json")))
    n = meta["n"]
    res = {}
    for name, v in meta["variants"].items():
        res[name] = _time(os.path.join(a.dir, v["lib"]), n, a.passes, meta.get("batch", 1))
        print(f"[autotune] {name:22s} {res[name]:.4f} ms/pass", flush=True)
    base = meta["base"]
    choice = dict(base)
    for k in SIZE_KNOBS[n]:
        best_v, best_t = base[k], res["base"]
        for name, t in res.items():
            if name.startswith(k + "=") and t < best_t:
                best_v, best_t = int(name.split("=")[1]), t
        choice[k] = best_v
    meta["times"] = res
    meta["choice"] = choice
    json.dump(meta, open(os.path.join(a.dir, "result.json"), "w"), indent=1)
    print(json.dumps({"choice": choice, "base_ms": res["base"]}), flush=True)


def other_knobs():
    """Knobs in recon_tuning.h that this tuner does not time (the deposit's launch shapes, timed on the
    survey catalogues), with the comment lines that record their timings: kept as they are."""
    text = open(TUNING).read()
    lines = text.splitlines()
    keep = []
    for i, l in enumerate(lines):         # the comment block that opens with "// Deposit"
        if l.startswith("// Deposit"):
            j = i
            while j < len(lines) and lines[j].startswith("//"):
                keep.append(lines[j])
                j += 1
            break
    for k, v in re.findall(r"#define\s+(RECON_\w+)\s+(\d+)", text):
        if k not in KNOBS:
            keep += [f"#ifndef {k}", f"#define {k} {v}", "#endif"]
    return keep


def size_blocks():
    """The timing comment block of each size, as written by the last tuning at that size."""
    blocks, cur = {}, None
    for l in open(TUNING).read().splitlines():
        m = re.match(r"// Chosen on a (\d+)\^3", l)
        if m:
            cur = int(m.group(1))
            blocks[cur] = [l]
        elif cur is not None and l.startswith("//   "):
            blocks[cur].append(l)
        else:
            cur = None
    return blocks


def cmd_write(a):
    meta = json.load(open(os.path.join(a.dir, "result.json")))
    choice, res, n = meta["choice"], meta["times"], meta["n"]
    if "combined_ms" in meta and meta["combined_ms"] >= res["base"]:
        choice = meta["base"]
        note = f"single-knob winners combined were not faster ({meta['combined_ms']:.4f} ms); kept"
    else:
        note = "fastest per knob"
    values = current()
    for k in SIZE_KNOBS[n]:
        values[k] = choice[k]
    blocks = size_blocks()
    batch = meta.get("batch", 1)
    blocks[n] = [f"// Chosen on a {n}^3 correction pass" + (f" of a batch of {batch}" if batch > 1 else "") +
                 f" ({note}); ms per pass of each variant:"]
    for name, t in sorted(res.items(), key=lambda kv: kv[1]):
        blocks[n].append(f"//   {name:22s} {t:.4f}")
    lines = ["// Tuning knobs of the transform kernels, written by paper_1504_02591_amd/autotune.py (a -D on the",
             "// compiler command line overrides them).  Tiles: packed z column pairs, y-pass columns, x-pass",
             "// rows per block; middle radix split of the 512- and 1024-point transforms; z tiles per block of",
             "// the z iteration; wave-local z iteration at 512^3.  The general knobs are timed at 512^3 and",
             "// serve every size without its own; the _256 and _1024 knobs are timed at those sizes."]
    for size in sorted(blocks):
        lines += blocks[size]
    lines.append("#pragma once")
    for k in KNOBS:
        lines += [f"#ifndef {k}", f"#define {k} {values[k]}", "#endif"]
    lines += other_knobs()
    open(TUNING, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_combined(a):
    """Build and time the combined choice (host build, then GPU timing)."""
    meta = json.load(open(os.path.join(a.dir, "result.json")))
    lib = os.path.join(a.dir, "lib_combined.so")
    if a.stage in ("build", "both"):
        _build_one(("combined", meta["choice"], lib))
    if a.stage in ("time", "both"):
        meta["combined_ms"] = _time(lib, meta["n"], a.passes, meta.get("batch", 1))
        json.dump(meta, open(os.path.join(a.dir, "result.json"), "w"), indent=1)
        print(json.dumps({"combined_ms": meta["combined_ms"], "base_ms": meta["times"]["base"]}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--dir", required=True)
    b.add_argument("--n", type=int, default=512, choices=sorted(SIZE_KNOBS))
    b.add_argument("--batch", type=int, default=1, help="realisations per plan in the timed passes")
    b.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    t = sub.add_parser("time")
    t.add_argument("--dir", required=True)
    t.add_argument("--passes", type=int, default=10)
    o = sub.add_parser("one")
    o.add_argument("--lib", required=True)
    o.add_argument("--n", type=int, default=512)
    o.add_argument("--passes", type=int, default=10)
    o.add_argument("--batch", type=int, default=1)
    o.add_argument("--field-cache", default=None, help="directory holding the drawn field between variants")
    c = sub.add_parser("combined")
    c.add_argument("--dir", required=True)
    c.add_argument("--stage", choices=["build", "time", "both"], default="both")
    c.add_argument("--passes", type=int, default=10)
    w = sub.add_parser("write")
    w.add_argument("--dir", required=True)
    a = ap.parse_args()
    {"build": cmd_build, "time": cmd_time, "one": cmd_one, "write": cmd_write, "combined": cmd_combined}[a.cmd](a)


if __name__ == "__main__":
    main()
