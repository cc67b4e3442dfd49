"""The tuner's measured table (paper_2507_04786_amd/csrc/tune_table.inc) and
the rule that emits it from sweep records (paper_2507_04786_amd/tune_sweep.py):
the table covers every (ranks, collective, size) the planner looks up, its
plans are legal (tree only for AllReduce, Section V-A), and the emit rule
takes the fastest plan, preferring fewer channels within its tolerance."""
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2507_04786_amd", "csrc", "tune_table.inc")
sys.path.insert(0, os.path.join(ROOT, "paper_2507_04786_amd"))
import tune_sweep as ts  # noqa: E402

ROW = re.compile(r"^\{(\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+), ([\d.]+)\},$")


def _rows():
    out = []
    for line in open(TABLE):
        line = line.strip()
        if not line or line.startswith("//"):
            continue
        m = ROW.match(line)
        assert m, f"malformed table row: {line}"
        R, coll, lg, algo, proto, C, chunk_kib, threads = (int(x) for x in m.groups()[:8])
        out.append(dict(R=R, coll=coll, lg=lg, algo=algo, proto=proto, C=C, chunk_kib=chunk_kib,
                        threads=threads, us=float(m.group(9))))
    return out


def test_table_covers_every_lookup():
    rows = _rows()
    keys = {(r["R"], r["coll"], r["lg"]) for r in rows}
    assert len(keys) == len(rows), "duplicate (ranks, collective, size) entries"
    for R in (4, 8, 16):
        for coll in range(5):
            sizes = sorted(lg for (r, c, lg) in keys if r == R and c == coll)
            assert sizes, (R, coll)
            # contiguous up to 256 MiB; AllGather / ReduceScatter start where
            # a block holds at least one fp32 element
            assert sizes == list(range(sizes[0], 29)), (R, coll, sizes)
            assert sizes[0] <= 3 + (R.bit_length() - 1 if coll in (3, 4) else 0), (R, coll, sizes[0])


def test_table_plans_are_legal():
    for r in _rows():
        assert r["algo"] in (0, 1) and r["proto"] in (0, 1, 2), r
        if r["algo"] == 1:
            assert r["coll"] == 0, f"tree only for AllReduce: {r}"
        assert r["C"] in ts.CHANNELS, r
        # chunk and threads are those the measured plan ran with: a swept
        # value or the planner's formula (chunks of 4 KiB granules up to the
        # Simple slot of the plan's connections, 256 KiB ring / 128 KiB
        # tree; workgroups of whole waves)
        if r["chunk_kib"]:
            assert r["proto"] == 0 and r["lg"] >= ts.CHUNK_MIN_LOG2, r
            assert r["chunk_kib"] % 4 == 0 and 16 <= r["chunk_kib"] <= (128 if r["algo"] == 1 else 256), r
        if r["threads"]:
            assert r["lg"] >= (ts.CHUNK_MIN_LOG2 if r["proto"] == 0 else ts.THREADS_MIN_LOG2), r
            assert r["threads"] % 64 == 0 and 64 <= r["threads"] <= 1024, r
        assert r["us"] > 0, r


def _rec(lg, C, ms, proto="simple", algo="ring", chunk=0, threads=0, ran_chunk=128 << 10):
    """A sweep record; a request of 0 ran with `ran_chunk` (the formula's, or
    the chunk of the table the library was built with) and the formula's
    workgroup (256 threads for Simple, 512 for LL / LL128 at these sizes)."""
    return dict(R=8, coll="allreduce", S=1 << lg, log2=lg, algo=algo, proto=proto, C=C, chunkReq=chunk, Treq=threads,
                Cplan=C, chunk=chunk or ran_chunk, T=threads or (256 if proto == "simple" else 512), direct=1, ms=ms,
                wall_ms=ms, reps=3)


def test_emit_prefers_fewer_channels_within_tolerance(tmp_path):
    small, large = 20, ts.LARGE_LOG2
    recs = [
        # below 16 MiB: 8 channels are 9 % slower than 32 -> within 10 %, taken
        _rec(small, 32, 1.00), _rec(small, 8, 1.09), _rec(small, 4, 1.20),
        # from 16 MiB: 16 channels 5 % slower -> outside 3 %, the fastest wins
        _rec(large, 32, 1.00, chunk=64 << 10), _rec(large, 16, 1.05), _rec(large, 8, 1.02, proto="ll", threads=1024),
    ]
    src = tmp_path / "sweep.jsonl"
    src.write_text("\n".join(json.dumps(r) for r in recs) + "\n")
    dest = tmp_path / "table.inc"
    ts.emit([str(src)], str(dest))
    rows = [ROW.match(line.strip()).groups() for line in open(dest) if line.startswith("{")]
    got = {int(r[2]): r for r in rows}
    assert got[small][3:8] == ("0", "0", "8", "128", "256")  # ring Simple, 8 channels, the chunk it ran
    assert got[large][3:8] == ("0", "1", "8", "0", "1024")  # LL at 8 channels: within 3 %, fewer
    # without the LL point the 32-channel plan with its 64 KiB chunk wins
    src.write_text("\n".join(json.dumps(r) for r in recs if r["proto"] == "simple") + "\n")
    ts.emit([str(src)], str(dest))
    rows = [ROW.match(line.strip()).groups() for line in open(dest) if line.startswith("{")]
    got = {int(r[2]): r for r in rows}
    assert got[large][3:8] == ("0", "0", "32", "64", "256")


def test_emit_uses_the_chunk_a_default_request_ran_with(tmp_path):
    """A request of chunk 0 resolves to the table the library was built
    with: a record that asked for 0 but ran with 32 KiB is the same plan as
    one that asked for 32 KiB, is averaged with it, and is emitted as
    32 KiB, not as the formula's chunk."""
    lg = 26
    recs = [_rec(lg, 32, 0.41, chunk=0, ran_chunk=32 << 10), _rec(lg, 32, 0.43, chunk=32 << 10),
            _rec(lg, 32, 0.46, chunk=64 << 10)]
    src = tmp_path / "sweep.jsonl"
    src.write_text("\n".join(json.dumps(r) for r in recs) + "\n")
    dest = tmp_path / "table.inc"
    ts.emit([str(src)], str(dest))
    rows = [ROW.match(line.strip()).groups() for line in open(dest) if line.startswith("{")]
    assert len(rows) == 1
    assert rows[0][3:8] == ("0", "0", "32", "32", "256")
    assert float(rows[0][8]) == 420.0  # the two runs of that plan averaged
