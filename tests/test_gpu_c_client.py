"""The library driven from plain C through include/vccl.h (tests/c_client.c):
AllReduce, grouped AllGather + ReduceScatter and Broadcast on int32 data,
checked inside the program against sums written out in C (exact in any
order), and the per-call cost of an 8-byte AllReduce issued from C."""
import json
import subprocess

import pytest

from tests import c_client_build as cb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    why = cb.available()
    if why:
        pytest.fail(why)
    out = tmp_path_factory.mktemp("c_client") / "c_client"
    cb.build(str(out))
    return str(out)


@pytest.mark.parametrize("R,n", [(4, 100003), (8, 4099), (16, 1), (2, 65536)])
def test_c_client(client, R, n):
    print(f"c_client R={R} n={n}", flush=True)
    res = subprocess.run([client, str(R), str(n)], capture_output=True, text=True, timeout=90)
    assert res.returncode == 0, f"exit {res.returncode}\n{res.stdout}\n{res.stderr}"
    line = [l for l in res.stdout.splitlines() if l.startswith("{")][-1]
    rec = json.loads(line)
    assert rec["ok"] == 1 and rec["nranks"] == R and rec["count"] == n
    print(line, flush=True)


def test_exit_with_live_sets_is_clean(client):
    """The same program leaves its communicator set and buffers alive and
    returns from main: the process still exits with status 0 (the library
    runs no code of its own at exit, so nothing of it touches the HIP
    runtime while the runtime tears down)."""
    res = subprocess.run([client, "8", "4099", "keep"], capture_output=True, text=True, timeout=90)
    assert res.returncode == 0, f"exit {res.returncode}\n{res.stdout}\n{res.stderr}"
    rec = json.loads([l for l in res.stdout.splitlines() if l.startswith("{")][-1])
    assert rec["ok"] == 1


@pytest.mark.parametrize("R,n", [(8, 50021), (5, 777)])
def test_c_client_on_ring_orders(client, R, n):
    """The same checks on a set created from C with two ring orders."""
    res = subprocess.run([client, str(R), str(n), "rings"], capture_output=True, text=True, timeout=90)
    assert res.returncode == 0, f"exit {res.returncode}\n{res.stdout}\n{res.stderr}"
    rec = json.loads([l for l in res.stdout.splitlines() if l.startswith("{")][-1])
    assert rec["ok"] == 1 and rec["nranks"] == R
