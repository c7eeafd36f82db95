"""Per-kernel HBM traffic from two rocprofv3 --pmc databases (FETCH_SIZE,
WRITE_SIZE in KiB per dispatch), scaled by what the same counters read for
a device copy of known size in the same run.

``python -m paper_2606_23031_amd.pmcsummary <fetch.db> <write.db> <bytes>``
prints JSON: per kernel the mean calibrated bytes per dispatch."""
import collections
import json
import sqlite3
import sys


def _per_kernel(db, counter):
    con = sqlite3.connect(db)
    out = collections.defaultdict(list)
    for name, val in con.execute(
            "select name, counter_value from pmc_events where counter_name=?",
            (counter,)):
        out[name.split("(")[0].replace("void ", "")].append(val)
    return out


def summary(fetch_db, write_db, copy_bytes):
    f = _per_kernel(fetch_db, "FETCH_SIZE")
    w = _per_kernel(write_db, "WRITE_SIZE")
    # the calibration copy is the last device-to-device copy of each run
    cf = f["__amd_rocclr_copyBuffer"][-1] * 1024.0
    cw = w["__amd_rocclr_copyBuffer"][-1] * 1024.0
    kf, kw = copy_bytes / cf, copy_bytes / cw
    res = {"copy_bytes": copy_bytes, "fetch_scale": kf, "write_scale": kw,
           "kernels": {}}
    for k in sorted(set(f) | set(w)):
        if not k.startswith("dv::"):
            continue
        fb = sum(f.get(k, [0])) / max(len(f.get(k, [])), 1) * 1024.0 * kf
        wb = sum(w.get(k, [0])) / max(len(w.get(k, [])), 1) * 1024.0 * kw
        res["kernels"][k] = {"fetch_bytes": fb, "write_bytes": wb}
    return res


if __name__ == "__main__":
    print(json.dumps(summary(sys.argv[1], sys.argv[2], float(sys.argv[3])),
                     indent=1))
