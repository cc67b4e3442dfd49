"""Line formats of the LL and LL128 protocols and the slot geometry of all
three protocols (Section III; Section V-C buffer table).

* LL (Section III-B): each transmission is 4 bytes of data followed by a
  4-byte flag, written together as one 8-byte unit.  Layout adopted: the
  unit is a little-endian 64-bit word, data in bytes 0..3, flag in bytes
  4..7.  A payload whose length is not a multiple of 4 is zero-padded in its
  last unit.
* LL128 (Section III-C): 128-byte units carrying 120 bytes of data and an
  8-byte flag.  Layout adopted: payload in bytes 0..119, the flag as a
  little-endian 64-bit word in bytes 120..127; a short last line is
  zero-padded.
* Flag values: the flag of the data sent in connection step ``s`` (0-based,
  counted over the connection's lifetime) is ``s + 1`` -- its low 32 bits
  for LL, the full 64 bits for LL128 -- so a slot's stale lines never carry
  the flag the receiver waits for.
* Slots: a channel buffer is split into ``slots`` equal slots (8 by
  default).  Slot capacities: Simple 512 KiB, LL 32 KiB, LL128 600 KiB; the
  data a slot carries per step is its capacity times the payload fraction
  (1, 1/2, 120/128).
"""
from __future__ import annotations

import numpy as np

SLOTS = 8
SLOT_BYTES = {"simple": 512 * 1024, "ll": 32 * 1024, "ll128": 600 * 1024}
LL_UNIT = 8
LL_DATA = 4
LL128_LINE = 128
LL128_DATA = 120


def payload_fraction(proto: str) -> float:
    return {"simple": 1.0, "ll": LL_DATA / LL_UNIT, "ll128": LL128_DATA / LL128_LINE}[proto]


def slot_payload_bytes(proto: str) -> int:
    cap = SLOT_BYTES[proto]
    if proto == "simple":
        return cap
    if proto == "ll":
        return cap // LL_UNIT * LL_DATA
    return cap // LL128_LINE * LL128_DATA


def channel_buffer_bytes(proto: str, slots: int = SLOTS) -> int:
    return SLOT_BYTES[proto] * slots


def ll_encode(payload: bytes | np.ndarray, step: int) -> np.ndarray:
    """Payload bytes -> array of 64-bit LL units carrying flag (step+1) mod 2^32."""
    b = np.frombuffer(bytes(payload), dtype=np.uint8) if not isinstance(payload, np.ndarray) else payload.view(np.uint8)
    nunits = -(-len(b) // LL_DATA)
    padded = np.zeros(nunits * LL_DATA, dtype=np.uint8)
    padded[:len(b)] = b
    data = padded.view("<u4").astype(np.uint64)
    flag = np.uint64((step + 1) & 0xFFFFFFFF)
    return data | (flag << np.uint64(32))


def ll_decode(units: np.ndarray, step: int, nbytes: int) -> tuple[np.ndarray, bool]:
    """Returns (payload bytes, all flags equal to the step's flag)."""
    units = np.asarray(units, dtype=np.uint64)
    flags = (units >> np.uint64(32)).astype(np.uint32)
    ok = bool((flags == np.uint32((step + 1) & 0xFFFFFFFF)).all())
    data = (units & np.uint64(0xFFFFFFFF)).astype("<u4").view(np.uint8)
    return data[:nbytes].copy(), ok


def ll128_encode(payload: bytes | np.ndarray, step: int) -> np.ndarray:
    """Payload bytes -> uint8 array of 128-byte lines, flag step+1 in bytes 120..127."""
    b = np.frombuffer(bytes(payload), dtype=np.uint8) if not isinstance(payload, np.ndarray) else payload.view(np.uint8)
    nlines = -(-len(b) // LL128_DATA)
    out = np.zeros((nlines, LL128_LINE), dtype=np.uint8)
    padded = np.zeros(nlines * LL128_DATA, dtype=np.uint8)
    padded[:len(b)] = b
    out[:, :LL128_DATA] = padded.reshape(nlines, LL128_DATA)
    out[:, LL128_DATA:] = np.array([step + 1], dtype="<u8").view(np.uint8)
    return out.reshape(-1)


def ll128_decode(lines: np.ndarray, step: int, nbytes: int) -> tuple[np.ndarray, bool]:
    arr = np.asarray(lines, dtype=np.uint8).reshape(-1, LL128_LINE)
    flags = arr[:, LL128_DATA:].copy().view("<u8").reshape(-1)
    ok = bool((flags == np.uint64(step + 1)).all())
    data = arr[:, :LL128_DATA].reshape(-1)
    return data[:nbytes].copy(), ok
