"""Tune the automatic launch shapes of mrg_generate on this GPU.

    python -m paper_2201_06604_amd.tune_plain            # time and print the table
    python -m paper_2201_06604_amd.tune_plain --write    # also rewrite csrc/mrg_tuned.h

csrc/mrg_tuned.h holds one entry per output kind and size class: streams per
lane, threads per block, the waves a grid aims at (which sets the chunk of
draws per work-item), the shortest chunk, lockstep rows and XCD block order.
For each kind and class this script creates the class's representative
workload (the stream count and draws per stream listed in the header, streams
created on the device from a fixed seed), works out the launch shape each
candidate entry resolves to under the automatic plan's rules (`resolve`, the
same steps plan_generate takes), times every distinct shape with mrg_generate_ex
(HIP events, median of 7 runs after a warm-up), and keeps the entry of the
fastest shape; the current entry stays unless another is faster by more than
2%.  The library must be rebuilt after --write.  Results never depend on the
shapes, only times do.
"""
import argparse
import os
import re
import sys

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(PKG, "csrc", "mrg_tuned.h")

UNIFORM, NORMAL, EXPONENTIAL, RAW = 0, 1, 2, 3
F64, F32, U32 = 0, 1, 2
KINDS = [("uniform f64", UNIFORM, F64), ("uniform f32", UNIFORM, F32), ("raw u32", RAW, U32),
         ("normal f64", NORMAL, F64), ("normal f32", NORMAL, F32), ("exponential f64", EXPONENTIAL, F64),
         ("exponential f32", EXPONENTIAL, F32)]
CLASSES = [(256, 256), (1024, 1024), (16384, 1024), (65536, 4096), (262144, 4096)]  # streams x draws
FIELDS = ("spl", "block", "waves", "min_units", "lock", "xcd")


def read_table(path=HEADER):
    """The entries of csrc/mrg_tuned.h as [kind][class] dicts."""
    src = open(path).read()
    body = src[src.index("kTuned[kTunedKinds][kTunedClasses] = {"):]
    nums = [tuple(int(v) for v in m.split(",")) for m in re.findall(r"\{(\s*\d+(?:\s*,\s*\d+){5})\s*\}", body)]
    assert len(nums) == len(KINDS) * len(CLASSES), len(nums)
    return [[dict(zip(FIELDS, nums[k * len(CLASSES) + c])) for c in range(len(CLASSES))]
            for k in range(len(KINDS))]


def write_table(table, notes, path=HEADER):
    src = open(path).read()
    cut = src.find("// Timings of the tuning run")
    head = src[:cut if cut >= 0 else src.index("// clang-format off")]
    tail = src[src.index("// clang-format on"):]
    rows = []
    for k, (name, _, _) in enumerate(KINDS):
        ents = ", ".join("{" + ", ".join(str(table[k][c][f]) for f in FIELDS) + "}" for c in range(len(CLASSES)))
        rows.append(f"    {{{ents}}},  // {name}")
    body = ("// clang-format off\n"
            "constexpr TunedShape kTuned[kTunedKinds][kTunedClasses] = {\n" + "\n".join(rows) + "\n};\n")
    note = "".join(f"// {ln}\n" for ln in notes)
    with open(path, "w") as f:
        f.write(head + note + body + tail)


def resolve(entry, S, n, dist, dtype):
    """The launch shape plan_generate gives an automatic call with this table
    entry (output aligned to 256 bytes): the keys of mrg_launch_cfg."""
    esz = 8 if dtype == F64 else 4
    spl = entry["spl"]
    while spl * esz > 16:
        spl //= 2
    while spl > 1 and S % spl:
        spl //= 2
    while spl > 1 and 64 * spl > S:
        spl //= 2
    q, r = divmod(n, S)
    cnt_max = q + (1 if r else 0)
    units_max = (cnt_max + 1) // 2 if dist == NORMAL else cnt_max
    n_sblk = -(-S // (64 * spl))
    w = -(-entry["waves"] // n_sblk)
    w = min(w, -(-units_max // entry["min_units"]))
    w = max(w, 1)
    chunk = max(1, -(-units_max // w))
    nch = -(-units_max // chunk) if units_max else 0
    if nch > 65535:
        chunk = -(-units_max // 65535)
        nch = -(-units_max // chunk)
    lock = 1 if entry["lock"] and n_sblk * nch >= 2048 else 0
    xcd = entry["xcd"]
    gx = -(-n_sblk // (entry["block"] // 64))
    if xcd and (gx * nch) % 8:
        xcd = 0
    return {"block": entry["block"], "chunk": chunk, "nontemporal": 1 if (S * esz) % 128 == 0 else 0,
            "arith": 2, "streams_per_lane": spl, "xcd_remap": xcd, "lockstep": lock}


def candidates(dist, dtype):
    spls = (1, 4) if dtype != F64 and dist in (UNIFORM, RAW) else (1, 2)
    locks = (0, 1) if (dist, dtype) == (UNIFORM, F64) else (0,)
    for spl in spls:
        for block in (256, 512):
            for waves in (1024, 2048, 4096, 8192, 16384):
                for min_units in (32, 96):
                    for lock in locks:
                        for xcd in (0, 1):
                            yield dict(spl=spl, block=block, waves=waves, min_units=min_units, lock=lock, xcd=xcd)


def tune(reps=7, verbose=True):
    import torch

    import paper_2201_06604_amd as P
    table = read_table()
    new = [[dict(e) for e in row] for row in table]
    notes = []
    torch.cuda.set_device(0)
    seed = [1234567, 7654321, 1111111, 2222222, 3333333, 4444444]
    for c, (S, per) in enumerate(CLASSES):
        n = S * per
        streams = P.mrg_streams_create_device(P.mrg_creator_init(seed), S)
        for k, (name, dist, dtype) in enumerate(KINDS):
            out = P.new_output(n, dtype)
            shapes = {}
            for cand in [table[k][c]] + list(candidates(dist, dtype)):
                key = tuple(sorted(resolve(cand, S, n, dist, dtype).items()))
                shapes.setdefault(key, cand)
            times = {}
            for key in shapes:
                cfg = dict(key)
                for _ in range(2):
                    P.mrg_generate(streams, n, dist, dtype, 1.0, out=out, cfg=cfg)
                ts = []
                for _ in range(reps):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    P.mrg_generate(streams, n, dist, dtype, 1.0, out=out, cfg=cfg)
                    b.record()
                    torch.cuda.synchronize()
                    ts.append(a.elapsed_time(b))
                times[key] = float(np.median(ts))
            cur = tuple(sorted(resolve(table[k][c], S, n, dist, dtype).items()))
            best = min(times, key=times.get)
            keep = times[cur] <= 1.02 * times[best]
            chosen = cur if keep else best
            new[k][c] = dict(table[k][c]) if keep else dict(shapes[best])
            line = (f"{name}, {S} x {per}: {times[chosen] * 1e3:.1f} us "
                    f"(entry before: {times[cur] * 1e3:.1f} us; {len(times)} shapes timed)")
            notes.append(line)
            if verbose:
                print(line, dict(chosen), flush=True)
            del out
        del streams
        torch.cuda.empty_cache()
    return new, notes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true", help="rewrite csrc/mrg_tuned.h with the result")
    ap.add_argument("--out", default=HEADER, help="where --write puts the header (default: csrc/mrg_tuned.h)")
    ap.add_argument("--reps", type=int, default=7)
    a = ap.parse_args()
    table, notes = tune(a.reps)
    if a.write:
        if a.out != HEADER:
            with open(a.out, "w") as f:
                f.write(open(HEADER).read())
        write_table(table, ["Timings of the tuning run that wrote this table (MI355X, median of "
                            f"{a.reps} launches):"] + notes, path=a.out)
        print("wrote", a.out)


if __name__ == "__main__":
    sys.exit(main())
