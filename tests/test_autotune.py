"""Host logic of the batched-engine autotuner: the table it writes and the
order in which the library reads it (the first row whose bounds hold)."""
import re

from paper_2108_05345_amd import autotune


def _lookup(rows, per_cu, mmax):
    # the rule of batch_engine() in the library, on the rows as written
    for r in rows + [{"per_cu_hi": 1e300, "m_hi": 1 << 30, "engine": 0}]:
        if per_cu <= r["per_cu_hi"] and mmax <= r["m_hi"]:
            return r["engine"]


def _cells():
    out = []
    best = {(0.5, 64): "fused", (0.5, 256): "phased", (2.0, 64): "fused2", (2.0, 256): "phased",
            (8.0, 64): "fused2"}
    for (pc, m), b in best.items():
        out.append({"per_cu": pc, "m": m, "best": b})
    return out


def test_rows_are_ordered_for_the_first_match_rule():
    rows = autotune.table_rows(_cells())
    keys = [(r["per_cu_hi"], r["m_hi"]) for r in rows]
    assert keys == sorted(keys)
    # a shape at or below a measured cell takes that cell's engine
    assert _lookup(rows, 0.3, 50) == 0
    assert _lookup(rows, 0.5, 200) == 2
    assert _lookup(rows, 1.5, 64) == 1
    assert _lookup(rows, 1.5, 100) == 2
    assert _lookup(rows, 6.0, 64) == 1
    # beyond every measured cell: the fused default
    assert _lookup(rows, 6.0, 100) == 0
    assert _lookup(rows, 20.0, 64) == 0


def test_header_lists_the_rows_in_order():
    rows = autotune.table_rows(_cells())
    text = autotune.header_text(rows, "test device")
    got = re.findall(r"\{([0-9.e+]+), (\d+|1 << 30), (\d)\},", text)
    assert [(float(a), b, int(c)) for a, b, c in got[:-1]] == [
        (r["per_cu_hi"], str(r["m_hi"]), r["engine"]) for r in rows]
    assert got[-1] == ("1e300", "1 << 30", "0")
    assert "kTuneRows" in text and text.count("namespace lhdm") == 2
