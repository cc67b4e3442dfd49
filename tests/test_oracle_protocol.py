"""Pins of the oracle's line formats and slot geometry against the paper's
tables (tests/golden/buffers_and_lines.txt)."""
import os

import numpy as np
import pytest

from oracle import protocol as pr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    out = {}
    for line in open(os.path.join(GOLDEN, "buffers_and_lines.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            out[k] = int(v)
    return out


def test_slot_geometry_matches_paper_table():
    g = _golden()
    assert pr.SLOTS == g["slots"]
    for proto in ("simple", "ll", "ll128"):
        assert pr.channel_buffer_bytes(proto) == g[f"{proto}.total"]
        assert pr.SLOT_BYTES[proto] == g[f"{proto}.slot"]
        assert pr.slot_payload_bytes(proto) == g[f"{proto}.payload"]


def test_line_payload_fractions():
    g = _golden()
    assert pr.payload_fraction("ll") == g["ll.line.data"] / (g["ll.line.data"] + g["ll.line.flag"]) == 0.5
    assert pr.payload_fraction("ll128") == g["ll128.line.data"] / (g["ll128.line.data"] + g["ll128.line.flag"])
    assert pr.payload_fraction("ll128") == 0.9375
    assert pr.LL_UNIT == g["ll.line.data"] + g["ll.line.flag"]
    assert pr.LL128_LINE == g["ll128.line.data"] + g["ll128.line.flag"]


@pytest.mark.parametrize("nbytes", [0, 1, 4, 7, 120, 121, 4096, 16384])
@pytest.mark.parametrize("step", [0, 5, 2**32 - 1, 2**33 + 7])
def test_line_roundtrip(nbytes, step):
    rng = np.random.default_rng(nbytes + step % 1000)
    data = rng.integers(0, 256, nbytes, dtype=np.uint8)
    units = pr.ll_encode(data, step)
    assert len(units) == -(-nbytes // 4)
    back, ok = pr.ll_decode(units, step, nbytes)
    assert ok and np.array_equal(back, data)
    assert not pr.ll_decode(units, step + 1, nbytes)[1] or nbytes == 0
    lines = pr.ll128_encode(data, step)
    assert len(lines) == 128 * (-(-nbytes // 120))
    back, ok = pr.ll128_decode(lines, step, nbytes)
    assert ok and np.array_equal(back, data)
    assert not pr.ll128_decode(lines, step + 1, nbytes)[1] or nbytes == 0


def test_ll_unit_layout_is_data_then_flag():
    u = pr.ll_encode(bytes([1, 2, 3, 4]), 0x10)
    raw = u.astype("<u8").view(np.uint8)
    assert raw.tolist() == [1, 2, 3, 4, 0x11, 0, 0, 0]
    line = pr.ll128_encode(bytes(range(120)), 0x41)
    assert line[:120].tolist() == list(range(120))
    assert line[120:].tolist() == [0x42, 0, 0, 0, 0, 0, 0, 0]
