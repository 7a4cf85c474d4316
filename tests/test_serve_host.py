"""The request loop's admission and batching logic on the CPU, with its
simulated device (every launch finishes after its bytes at a fixed rate), so
no GPU is touched."""
import numpy as np
import pytest

import seedgen


@pytest.fixture(scope="module")
def A():
    from paper_1403_7295_amd import aesgpu
    return aesgpu


def requests(A, n, rate, seed=5, lo=64, hi=1 << 22):
    f, keys = seedgen.served_requests(seed, n, rate, lo=lo, hi=hi)
    r = np.zeros(n, A.REQUEST_DTYPE)
    for k, v in f.items():
        r[k] = v
    return r, keys


def test_all_complete_and_budget_holds(A):
    r, _ = requests(A, 3000, rate=50000.0)
    budget = 64 << 20
    cfg = A.serve_cfg(streams=4, budget_bytes=budget, max_batch_msgs=256, simulate_gbps=200.0)
    res, st = A.aes_serve_run(r, cfg)
    fp = 2 * ((r["nbytes"] + 255) // 256 * 256)
    big = fp > budget
    assert st["completed"] == (~big).sum() and st["rejected"] == big.sum()
    assert (res["status"][big] == A.AES_E_BUDGET).all()
    assert (res["status"][~big] == A.AES_OK).all()
    assert st["max_inflight_bytes"] <= budget
    ok = ~big
    assert (res["latency_s"][ok] > 0).all()
    assert (res["admit_s"][ok] >= 0).all()
    assert (res["latency_s"][ok] >= res["admit_s"][ok]).all()
    assert st["bytes_done"] == int(r["nbytes"][ok].sum())


def test_overload_runs_at_device_rate_and_batches(A):
    # offered ~10x the simulated device rate: the loop must batch and keep
    # the device busy, so completed bytes / span approaches the device rate
    r, _ = requests(A, 4000, rate=400000.0, hi=1 << 20)
    rate = 20.0
    cfg = A.serve_cfg(streams=4, budget_bytes=1 << 30, max_batch_msgs=512, simulate_gbps=rate)
    res, st = A.aes_serve_run(r, cfg)
    achieved = st["bytes_done"] / st["span_s"] / 1e9
    assert 0.8 * rate < achieved <= rate * 1.01
    assert st["launches"] < len(r) / 4          # many requests per launch
    lat = res["latency_s"]
    assert np.percentile(lat, 99) > np.percentile(lat, 50) > 0


def test_light_load_latency_is_service_time(A):
    r, _ = requests(A, 500, rate=2000.0, hi=1 << 16)
    cfg = A.serve_cfg(streams=4, budget_bytes=1 << 30, max_batch_msgs=64, simulate_gbps=100.0)
    res, st = A.aes_serve_run(r, cfg)
    service = r["nbytes"] / 100e9 + 20e-6
    # at 2,000 requests/s each request is nearly alone: latency is its own
    # service time plus loop overhead
    assert np.median(res["latency_s"] - service) < 200e-6
    assert st["completed"] == 500


def test_small_budget_makes_requests_wait(A):
    r, _ = requests(A, 400, rate=200000.0, lo=1 << 20, hi=1 << 20)
    budget = 8 * (2 << 20)                       # room for 8 requests at once
    cfg = A.serve_cfg(streams=2, budget_bytes=budget, max_batch_msgs=64, simulate_gbps=50.0)
    res, st = A.aes_serve_run(r, cfg)
    assert st["max_inflight_reqs"] <= 8 and st["max_inflight_bytes"] <= budget
    assert (res["admit_s"] > 1e-4).sum() > 100    # most requests queued for memory
    assert st["completed"] == 400


def test_argument_checks(A):
    r, _ = requests(A, 10, rate=1000.0)
    cfg = A.serve_cfg(simulate_gbps=10.0)
    bad = r.copy()
    bad["arrival_s"][3] = -1.0
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, cfg)
    assert e.value.code == A.AES_E_ARG
    bad = r.copy()
    bad["keybits_code"][0] = 3
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, cfg)
    assert e.value.code == A.AES_E_ARG
    bad = r.copy()
    bad["mode"][0] = 0
    bad["nbytes"][0] = 17
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, cfg)
    assert e.value.code == A.AES_E_LENGTH
    # a key slot of 2^31 or more must not pass as a negative int
    bad = r.copy()
    bad["key_idx"][2] = 1 << 31
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, cfg, nkeys=8)
    assert e.value.code == A.AES_E_ARG
    bad["key_idx"][2] = 8
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, cfg, nkeys=8)
    assert e.value.code == A.AES_E_ARG
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(r, cfg, nkeys=0)
    assert e.value.code == A.AES_E_ARG
    # CTR requests hold at most 2^36 bytes
    bad = r.copy()
    bad["mode"][1] = A.AES_MODE_CTR
    bad["nbytes"][1] = (1 << 36) + 16
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, A.serve_cfg(budget_bytes=1 << 40, simulate_gbps=10.0))
    assert e.value.code == A.AES_E_LENGTH
    for kw in ({"streams": 0}, {"streams": 17}, {"max_batch_msgs": 0}, {"budget_bytes": 100},
               {"blocks_per_thread": 3}):
        with pytest.raises(A.AESError) as e:
            A.aes_serve_scratch_size(A.serve_cfg(**kw))
        assert e.value.code == A.AES_E_ARG
    # without simulation a device is required: scratch must be given
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(r, A.serve_cfg())
    assert e.value.code == A.AES_E_NULL


def test_empty_run(A):
    res, st = A.aes_serve_run(np.zeros(0, A.REQUEST_DTYPE), A.serve_cfg(simulate_gbps=1.0))
    assert st["completed"] == 0 and len(res) == 0


def test_arena_is_not_reused_while_space_remains(A):
    # next-fit: with room for everything, no two requests share memory, even
    # though early requests finish (and free theirs) before late ones arrive
    r, _ = requests(A, 500, rate=100000.0, hi=1 << 18)
    fp = 2 * ((r["nbytes"].astype(np.int64) + 255) // 256 * 256)
    cfg = A.serve_cfg(streams=3, budget_bytes=int(fp.sum()), max_batch_msgs=16, simulate_gbps=50.0)
    res, st = A.aes_serve_run(r, cfg)
    assert st["completed"] == 500
    spans = sorted(zip(res["in_off"].tolist(), fp.tolist()))
    for (a, na), (b, _) in zip(spans, spans[1:]):
        assert a + na <= b


def _overwritten_by_later(A, r, res):
    """For every request, whether a request after it in arrival order (the
    loop admits in that order) was given memory overlapping its output."""
    fp = 2 * ((r["nbytes"].astype(np.int64) + 255) // 256 * 256)
    ok = res["status"] == A.AES_OK
    lo = res["in_off"].astype(np.int64)
    hi = lo + fp
    out_lo = res["out_off"].astype(np.int64)
    out_hi = out_lo + fp // 2
    n = len(r)
    want = np.zeros(n, bool)
    for i in range(n):
        if not ok[i] or fp[i] == 0:
            continue
        later = np.arange(n) > i
        later &= ok & (fp > 0)
        want[i] = bool(np.any(later & (lo < out_hi[i]) & (out_lo[i] < hi)))
    return want


@pytest.mark.parametrize("budget_mib", [4, 16, 64])
def test_overwritten_flags_name_exactly_the_reused_outputs(A, budget_mib):
    # a small arena forces reuse; every result the loop reports intact has
    # no later request over its output, and every reused one is flagged
    r, _ = requests(A, 1500, rate=100000.0, hi=1 << 20)
    cfg = A.serve_cfg(streams=3, budget_bytes=budget_mib << 20, max_batch_msgs=32, simulate_gbps=40.0)
    res, st = A.aes_serve_run(r, cfg)
    want = _overwritten_by_later(A, r, res)
    assert np.array_equal(res["overwritten"].astype(bool), want)
    assert want.any() and (~want & (res["status"] == A.AES_OK)).any()


def test_nothing_is_overwritten_with_room_for_everything(A):
    r, _ = requests(A, 400, rate=100000.0, hi=1 << 18)
    fp = 2 * ((r["nbytes"].astype(np.int64) + 255) // 256 * 256)
    cfg = A.serve_cfg(streams=3, budget_bytes=int(fp.sum()), max_batch_msgs=16, simulate_gbps=50.0)
    res, _ = A.aes_serve_run(r, cfg)
    assert not res["overwritten"].any()


def test_gcm_requests_take_16_more_bytes(A):
    # a GCM request's input and output each carry a 16-byte tag after the
    # data, counted against the budget; the simulated loop reports encryption
    # tags as written and decryptions (no device to check them) as not
    r, _ = requests(A, 300, rate=50000.0, hi=1 << 16)
    r["mode"] = A.AES_MODE_GCM
    budget = 1 << 22
    cfg = A.serve_cfg(streams=2, budget_bytes=budget, max_batch_msgs=16, simulate_gbps=40.0)
    res, st = A.aes_serve_run(r, cfg)
    fp = 2 * ((r["nbytes"].astype(np.int64) + 16 + 255) // 256 * 256)
    assert st["completed"] == 300 and st["max_inflight_bytes"] <= budget
    gap = res["out_off"].astype(np.int64) - res["in_off"].astype(np.int64)
    assert np.array_equal(gap, fp // 2)
    assert (res["authentic"] == np.where(r["decrypt"] == 1, 0, 1)).all()
    other, _ = requests(A, 50, rate=50000.0, hi=1 << 16)
    res2, _ = A.aes_serve_run(other, cfg)
    assert (res2["authentic"] == -1).all()


def test_gcm_request_checks(A):
    r, _ = requests(A, 10, rate=1000.0)
    bad = r.copy()
    bad["mode"][4] = A.AES_MODE_XTS          # not a served mode
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, A.serve_cfg(simulate_gbps=10.0))
    assert e.value.code == A.AES_E_ARG
    bad = r.copy()
    bad["mode"][4] = A.AES_MODE_GCM
    bad["nbytes"][4] = (1 << 36) - 16        # over GCM's 2^36 - 32
    with pytest.raises(A.AESError) as e:
        A.aes_serve_run(bad, A.serve_cfg(budget_bytes=1 << 40, simulate_gbps=10.0))
    assert e.value.code == A.AES_E_LENGTH
