"""Per-dispatch HBM traffic of the pass kernels (two passes and fused pass)
from two rocprofv3 --pmc runs of `bench.py --pmc-probe` (FETCH_SIZE, then
WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for
the probe's plain device copy of known size, per workload (CT 256x256,
radiotherapy).

Writes a JSON table keyed by kernel template, stamped with the SHA-256 of the
kernel source it was measured on (a changed kernel invalidates it).

    python pmc_summary.py FETCH_DB WRITE_DB OUT_JSON
"""
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2606_27086_amd")
COPY_BYTES = 512 * 1024 * 1024


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "smx_internal.h"):
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    return h.hexdigest()


CT_WORKLOAD = "ct256_parallel_beam_180x363_tv"
RT_WORKLOAD = "rt_160x160x80_9beams_47x47"


def dispatches(db: str, counter: str):
    con = sqlite3.connect(db)
    return con.execute(
        "select dispatch_id, kernel_name, value from counters_collection where counter_name = ? "
        "order by dispatch_id", (counter,)).fetchall()


def split(rows):
    """(reference copy KiB, {workload: {kernel: [KiB per dispatch]}}): the
    largest copy is the reference; dispatches after the marking copy belong to
    the radiotherapy workload, the ones before it to CT."""
    copies = [(d, v) for d, k, v in rows if "copyBuffer" in k]
    ref = max(v for d, v in copies)
    ref_id = max(copies, key=lambda c: c[1])[0]
    # the marking copy moves COPY_BYTES / 8 (the solver's own small copies are
    # far smaller)
    later = [d for d, v in copies if d > ref_id and 0.5 * ref / 8 < v < 2.0 * ref / 8]
    mark = min(later) if later else None
    out = {CT_WORKLOAD: {}, RT_WORKLOAD: {}}
    for d, k, v in rows:
        if "k_pass" not in k and "k_fused" not in k:
            continue
        wl = RT_WORKLOAD if (mark is not None and d > mark) else CT_WORKLOAD
        out[wl].setdefault(k.split("(")[0].replace("void ", ""), []).append(float(v))
    return ref, out


def summarise(fetch_db: str, write_db: str) -> dict:
    cf, f = split(dispatches(fetch_db, "FETCH_SIZE"))
    cw, w = split(dispatches(write_db, "WRITE_SIZE"))
    sf = COPY_BYTES / (cf * 1024.0)
    sw = COPY_BYTES / (cw * 1024.0)
    out = {"copy_bytes": COPY_BYTES, "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": sf,
           "write_scale": sw, "kernel_source_sha256": kernel_source_hash(), "workloads": {}}
    for wl in (CT_WORKLOAD, RT_WORKLOAD):
        ks = {}
        for name in sorted(set(f[wl]) | set(w[wl])):
            fb = sum(f[wl][name]) / len(f[wl][name]) * 1024.0 * sf if name in f[wl] else None
            wb = sum(w[wl][name]) / len(w[wl][name]) * 1024.0 * sw if name in w[wl] else None
            ks[name] = {"fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": (fb or 0.0) + (wb or 0.0),
                        "dispatches": len(f[wl].get(name, []))}
        out["workloads"][wl] = {"kernels": ks}
    return out


if __name__ == "__main__":
    res = summarise(sys.argv[1], sys.argv[2])
    with open(sys.argv[3], "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    print(json.dumps({k: v for k, v in res.items() if k != "kernels"}, indent=1))
