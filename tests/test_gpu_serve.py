"""The request loop on the GPU: payloads filled on the device match the
shared generator, and every request's result is the same alone (a single
aes_encrypt / aes_decrypt call on its own buffer) as in the mix of
overlapping batches (tolerance: zero bits), with and without arena reuse."""
import numpy as np
import pytest

import seedgen
from oracle import ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def A():
    from paper_1403_7295_amd import aesgpu
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return aesgpu


def requests(A, n, rate, seed, lo=64, hi=1 << 20):
    f, keys = seedgen.served_requests(seed, n, rate, lo=lo, hi=hi)
    r = np.zeros(n, A.REQUEST_DTYPE)
    for k, v in f.items():
        r[k] = v
    return r, keys


def alone(A, q, key, payload):
    """The request computed by itself through the single-buffer call."""
    bits = 128 + 64 * int(q["keybits_code"])
    rk, nr = A.aes_expand_key(key[:bits // 8])
    x = torch.from_numpy(payload).to("cuda")
    y = torch.empty_like(x)
    fn = A.aes_decrypt if q["decrypt"] else A.aes_encrypt
    mode = {0: "ecb", 1: "ctr", 2: "cbc"}[int(q["mode"])]
    fn(x, y, x.numel(), rk, nr, mode, ctr0=q["ctr0"])
    return y


def test_results_same_alone_and_in_the_mix(A):
    r, keys = requests(A, 300, rate=1e6, seed=51)
    fp = 2 * ((r["nbytes"].astype(np.int64) + 255) // 256 * 256)
    cfg = A.serve_cfg(streams=4, budget_bytes=int(fp.sum()) + (1 << 20), max_batch_msgs=32)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    torch.cuda.synchronize()
    assert st["completed"] == len(r) and st["rejected"] == 0
    assert st["launches"] > 4, "the requests should spread over several overlapping launches"
    o = ref.default()
    arena = srv.scratch
    for i, q in enumerate(r):
        n = int(q["nbytes"])
        payload = seedgen.bytes_np(int(q["payload_seed"]), n)
        i0 = int(res["in_off"][i])
        assert np.array_equal(arena[i0:i0 + n].cpu().numpy(), payload), "payload %d" % i
        got = srv.output(res[i], n)
        assert torch.equal(got, alone(A, q, keys[i], payload)), "request %d" % i
        if n <= 4096:
            bits = 128 + 64 * int(q["keybits_code"])
            rk, nr = o.expand_key(keys[i][:bits // 8])
            assert np.array_equal(got.cpu().numpy(), o.ctr(rk, nr, q["ctr0"], payload)), "oracle %d" % i


def test_results_with_arena_reuse(A):
    n = 256
    r, keys = requests(A, n, rate=2e6, seed=52, lo=65536, hi=65536)
    budget = 16 * 2 * 65536                      # 16 requests in flight at most
    cfg = A.serve_cfg(streams=3, budget_bytes=budget, max_batch_msgs=8)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    torch.cuda.synchronize()
    assert st["completed"] == n and st["max_inflight_bytes"] <= budget
    assert len(set(res["in_off"].tolist())) <= 16 < n
    # the last request to use each arena region still has its output there
    last = {}
    for i in range(n):
        off = int(res["in_off"][i])
        if off not in last or res["launch"][i] >= res["launch"][last[off]]:
            last[off] = i
    for off, i in last.items():
        payload = seedgen.bytes_np(int(r["payload_seed"][i]), 65536)
        assert torch.equal(srv.output(res[i], 65536), alone(A, r[i], keys[i], payload)), i


def test_latencies_are_consistent(A):
    r, keys = requests(A, 2000, rate=2e5, seed=53, hi=1 << 22)
    cfg = A.serve_cfg(streams=4, budget_bytes=1 << 30, max_batch_msgs=256)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    assert st["completed"] == 2000
    assert (res["latency_s"] > 0).all() and (res["latency_s"] >= res["admit_s"]).all()
    assert st["bytes_done"] == int(r["nbytes"].sum())


def test_mixed_modes_same_alone_and_in_the_mix(A):
    """ECB and CBC requests in both directions beside CTR ones: batches then
    use the inverse list (ECB and CBC decryption) and the serial one (CBC
    encryption) too, each launched only when a batch has such requests."""
    r, keys = requests(A, 200, rate=1e6, seed=54, hi=1 << 18)
    rng = np.random.default_rng(54)
    r["mode"] = rng.choice([0, 1, 2], len(r))
    r["decrypt"] = rng.integers(0, 2, len(r))
    whole = r["mode"] != 1
    r["nbytes"] = np.where(whole, np.maximum(r["nbytes"] // 16 * 16, 16), r["nbytes"])
    # room for every request, so that no output is overwritten before it is read
    fp = 2 * ((r["nbytes"].astype(np.int64) + 255) // 256 * 256)
    cfg = A.serve_cfg(streams=4, budget_bytes=int(fp.sum()) + (1 << 20), max_batch_msgs=16)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    torch.cuda.synchronize()
    assert st["completed"] == len(r) and st["rejected"] == 0 and st["launches"] > 4
    for i, q in enumerate(r):
        n = int(q["nbytes"])
        payload = seedgen.bytes_np(int(q["payload_seed"]), n)
        assert torch.equal(srv.output(res[i], n), alone(A, q, keys[i], payload)), "request %d (%s)" % (i, q)
