"""Per-dispatch HBM traffic of the pass kernels from two rocprofv3 --pmc runs
of pmc_probe.py (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
what the same counter reads for the probe's plain device copy of known size.

Writes a JSON table keyed by kernel template, stamped with the SHA-256 of the
kernel source it was measured on (a changed kernel invalidates it).

    python paper_2606_27086_amd/pmc_summary.py FETCH_DB WRITE_DB OUT_JSON
"""
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 512 * 1024 * 1024


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "smx_internal.h"):
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    return h.hexdigest()


def per_kernel(db: str, counter: str) -> dict:
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, avg(value), count(*), max(value) from counters_collection where counter_name = ? "
        "group by kernel_name", (counter,)).fetchall()
    return {r[0]: (float(r[1]), int(r[2]), float(r[3])) for r in rows}


def summarise(fetch_db: str, write_db: str) -> dict:
    f = per_kernel(fetch_db, "FETCH_SIZE")
    w = per_kernel(write_db, "WRITE_SIZE")
    # reference: the largest dispatch of the runtime's device-to-device copy kernel
    cf = max(v[2] for k, v in f.items() if "copyBuffer" in k)
    cw = max(v[2] for k, v in w.items() if "copyBuffer" in k)
    sf = COPY_BYTES / (cf * 1024.0)
    sw = COPY_BYTES / (cw * 1024.0)
    out = {"workload": "ct256_parallel_beam_180x363_tv", "copy_bytes": COPY_BYTES, "copy_fetch_kib": cf,
           "copy_write_kib": cw, "fetch_scale": sf, "write_scale": sw, "kernel_source_sha256": kernel_source_hash(),
           "kernels": {}}
    for name in sorted(set(f) | set(w)):
        if "k_pass" not in name:
            continue
        key = name.split("(")[0].replace("void ", "")
        fb = f[name][0] * 1024.0 * sf if name in f else None
        wb = w[name][0] * 1024.0 * sw if name in w else None
        out["kernels"][key] = {"fetch_bytes": fb, "write_bytes": wb,
                               "traffic_bytes": (fb or 0.0) + (wb or 0.0)}
    return out


if __name__ == "__main__":
    res = summarise(sys.argv[1], sys.argv[2])
    with open(sys.argv[3], "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    print(json.dumps({k: v for k, v in res.items() if k != "kernels"}, indent=1))
