"""The planner on the host, with no device (vcclDebugPlanHost): the LL128 gate
of Section III-C -- where LL128's 128-byte lines are not guaranteed whole,
no plan, tuned or requested, uses LL128 -- and the basic plan invariants the
kernels rely on."""
import pytest

COLLS = (0, 1, 2, 3, 4)
SIZES = [1 << k for k in range(3, 29, 1)]


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _count(coll, size, dtype_bytes, R):
    # the nccl-tests size convention: size is the larger per-rank buffer
    n = size // dtype_bytes
    if coll in (3, 4):
        n //= R
    return max(1, n)


def test_gate_off_never_plans_ll128(vccl):
    seen_ll128_when_on = 0
    for R in (4, 8, 16):
        for coll in COLLS:
            for S in SIZES:
                n = _count(coll, S, 2, R)
                on = vccl.vcclDebugPlanHost(R, coll, n, vccl.vcclBfloat16, ll128=1)
                off = vccl.vcclDebugPlanHost(R, coll, n, vccl.vcclBfloat16, ll128=0)
                assert on["ll128"] == 1 and off["ll128"] == 0
                assert off["proto"] != vccl.vcclProtoLL128, (R, coll, S, off)
                if on["proto"] == vccl.vcclProtoLL128:
                    seen_ll128_when_on += 1
                    # the fallback is the other flag protocol, with LL's slot-sized chunk
                    assert off["proto"] == vccl.vcclProtoLL, (R, coll, S, off)
                    assert off["chunkBytes"] <= 16 * 1024
                else:
                    assert off == dict(on, ll128=0), (R, coll, S)
    # the measured table does choose LL128 somewhere, so the gate is exercised
    assert seen_ll128_when_on > 0


def test_gate_off_overrides_an_explicit_ll128_request(vccl):
    t = dict(algo=vccl.vcclAlgoRing, proto=vccl.vcclProtoLL128, nchannels=8)
    on = vccl.vcclDebugPlanHost(8, 0, 1 << 20, vccl.vcclFloat32, ll128=1, tuning=t)
    off = vccl.vcclDebugPlanHost(8, 0, 1 << 20, vccl.vcclFloat32, ll128=0, tuning=t)
    assert on["proto"] == vccl.vcclProtoLL128 and on["nchannels"] == 8
    assert off["proto"] == vccl.vcclProtoLL and off["nchannels"] == 8


def test_plans_are_legal(vccl):
    """Every plan fits the model device and the slot it writes into:
    channels within the lane limit, chunk a multiple of 16 within the slot
    payload, workgroup size 64..1024 in steps of 64, a grid that is resident
    at once (1024 / nthreads workgroups per compute unit, 256 units), trees
    only for AllReduce."""
    # slot payloads of the ring and the tree connections, per protocol
    payload = {(0, 0): 256 * 1024, (0, 1): 16 * 1024, (0, 2): 4800 * 120,
               (1, 0): 128 * 1024, (1, 1): 16 * 1024, (1, 2): 1024 * 120}
    for R in (2, 3, 4, 7, 8, 12, 16):
        lanes = max(32, min(64, (2 * 256 // R) // 8 * 8))
        for coll in COLLS:
            for S in SIZES:
                for single in (0, 1):
                    p = vccl.vcclDebugPlanHost(R, coll, _count(coll, S, 4, R), vccl.vcclFloat32, single=single)
                    assert 1 <= p["nchannels"] <= lanes
                    assert p["chunkBytes"] % 16 == 0 and 16 <= p["chunkBytes"] <= payload[(p["algo"], p["proto"])]
                    assert 64 <= p["nthreads"] <= 1024 and p["nthreads"] % 64 == 0
                    assert p["grid"] <= 256 * max(1, 1024 // p["nthreads"])
                    assert p["grid"] == 8 * R * ((p["nlanes"] + 7) // 8)
                    if coll != 0:
                        assert p["algo"] == vccl.vcclAlgoRing


def test_rejects_bad_arguments(vccl):
    for args in ((1, 0, 8), (17, 0, 8), (8, 5, 8), (8, 0, 0)):
        with pytest.raises(vccl.VcclError) as e:
            vccl.vcclDebugPlanHost(args[0], args[1], args[2], vccl.vcclFloat32)
        assert e.value.code == vccl.vcclInvalidArgument
    with pytest.raises(vccl.VcclError):
        vccl.vcclDebugPlanHost(8, 0, 8, vccl.vcclFloat32, tuning=dict(nthreads=100))


def test_split_tree_fits_the_lane_limit(vccl):
    """A Simple tree launched alone runs as split halves on 8 ceil(C / 8) + C
    lanes, within the set's lane limit: 16 ranks (32 lanes) keep at most 16
    split channels, 8 ranks (64 lanes) up to 32; inside a group the channels
    stay fused, one lane each."""
    n = (64 << 20) // 2
    for R, asked, channels in ((16, 24, 16), (16, 16, 16), (8, 32, 32), (8, 24, 24), (8, 20, 20)):
        tune = dict(algo=vccl.vcclAlgoTree, proto=vccl.vcclProtoSimple, nchannels=asked)
        p = vccl.vcclDebugPlanHost(R, 0, n, vccl.vcclBfloat16, single=1, tuning=tune)
        assert p["algo"] == vccl.vcclAlgoTree and p["nchannels"] == channels, (R, asked, p)
        assert p["nlanes"] == 8 * ((channels + 7) // 8) + channels, (R, asked, p)
        assert p["nlanes"] <= max(32, min(64, (2 * 256 // R) // 8 * 8))
        g = vccl.vcclDebugPlanHost(R, 0, n, vccl.vcclBfloat16, single=0, tuning=tune)
        assert g["nlanes"] == g["nchannels"] == asked, (R, asked, g)
