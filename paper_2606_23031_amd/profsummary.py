"""Summarise a rocprofv3 kernel-trace database into a short Markdown table
(``python -m paper_2606_23031_amd.profsummary <results.db> "<command>"``)."""
import sqlite3
import sys


def summary(db, command, top=16):
    con = sqlite3.connect(db)
    cur = con.cursor()
    lines = [f"Command: `{command}`", "",
             "| kernel | calls | avg us | total us | % |",
             "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in cur.execute(
            "select name, total_calls, total_duration, average, percentage "
            f"from top_kernels limit {top}"):
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"| {short} | {calls} | {avg:.1f} | {tot:.1f} | {pct:.2f} |")
    lines += ["", "| kernel | VGPR | SGPR | LDS bytes | scratch |",
              "|---|---|---|---|---|"]
    seen = set()
    for r in cur.execute("select name, vgpr_count, sgpr_count, lds_size, "
                         "scratch_size from kernels"):
        short = r[0].split("(")[0].replace("void ", "")
        if short in seen or not short.startswith("dv::"):
            continue
        seen.add(short)
        lines.append(f"| {short} | {r[1]} | {r[2]} | {r[3]} | {r[4]} |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    print(summary(sys.argv[1], sys.argv[2]))
