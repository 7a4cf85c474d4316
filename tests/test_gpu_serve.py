"""The request loop on the GPU: payloads filled on the device match the
shared generator, and every request's result is the same alone (a single
aes_encrypt / aes_decrypt call on its own buffer) as in the mix of
overlapping batches (tolerance: zero bits), with and without arena reuse,
and equals the oracle's over the served workload's whole size range."""
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
    intact = set(np.nonzero(res["overwritten"] == 0)[0].tolist())
    assert set(last.values()) == intact
    # and every result the loop reports intact is that request's output
    for i in sorted(intact):
        payload = seedgen.bytes_np(int(r["payload_seed"][i]), 65536)
        assert torch.equal(srv.output(res[i], 65536), alone(A, r[i], keys[i], payload)), i


def oracle_check(O, q, key, out_dev, whole_limit=1 << 20, samples=64):
    """One served CTR request's output against the oracle: all of it up to
    whole_limit bytes, else the first and last (partial) blocks and
    `samples` blocks between them, each recomputed from its own counter."""
    n = int(q["nbytes"])
    bits = 128 + 64 * int(q["keybits_code"])
    rk, nr = O.expand_key(key[:bits // 8])
    seed = int(q["payload_seed"])
    if n <= whole_limit:
        want = O.ctr(rk, nr, q["ctr0"], seedgen.bytes_np(seed, n))
        return np.array_equal(out_dev.cpu().numpy(), want)
    nblk = (n + 15) // 16
    rng = np.random.default_rng(seed & 0xFFFFFFFF)
    idx = np.unique(np.concatenate([[0, nblk - 1], rng.integers(1, nblk - 1, samples)]))
    for j in idx.tolist():
        lo, hi = 16 * j, min(16 * j + 16, n)
        want = O.ctr(rk, nr, q["ctr0"], seedgen.bytes_np(seed, hi - lo, offset=lo), first_block=j)
        if not np.array_equal(out_dev[lo:hi].cpu().numpy(), want):
            return False
    return True


def test_served_workload_sizes_match_the_oracle(A):
    """Requests shaped like the served workload (CTR, AES-128/256, 70 %
    encryption, sizes log-uniform from 64 B to 64 MiB, byte-granular), with
    room for all of them in the arena so that every output can be read after
    the run: each equals the single-call result and the oracle's."""
    r, keys = requests(A, 400, rate=2e4, seed=55, lo=64, hi=1 << 26)
    assert r["nbytes"].max() > (32 << 20) and r["nbytes"].min() < 256
    fp = 2 * ((r["nbytes"].astype(np.int64) + 255) // 256 * 256)
    cfg = A.serve_cfg(streams=4, budget_bytes=int(fp.sum()) + (1 << 20), max_batch_msgs=64)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    torch.cuda.synchronize()
    assert st["completed"] == len(r) and st["rejected"] == 0 and st["launches"] > 4
    assert not res["overwritten"].any() and (res["status"] == A.AES_OK).all()
    o = ref.default()
    for i, q in enumerate(r):
        n = int(q["nbytes"])
        got = srv.output(res[i], n)
        assert oracle_check(o, q, keys[i], got), "oracle, request %d (%d bytes)" % (i, n)
        x = seedgen.bytes_torch(int(q["payload_seed"]), n, "cuda")
        y = torch.empty_like(x)
        fn = A.aes_decrypt if q["decrypt"] else A.aes_encrypt
        bits = 128 + 64 * int(q["keybits_code"])
        rk, nr = A.aes_expand_key(keys[i][:bits // 8])
        fn(x, y, n, rk, nr, "ctr", ctr0=q["ctr0"])
        assert torch.equal(got, y), "alone vs in the mix, request %d (%d bytes)" % (i, n)


def test_served_workload_with_reuse_intact_results_match_the_oracle(A):
    """The same shape under a budget a fraction of the total, so arena
    memory is reused: every result the loop reports intact is checked."""
    r, keys = requests(A, 400, rate=2e4, seed=56, lo=64, hi=1 << 26)
    cfg = A.serve_cfg(streams=4, budget_bytes=512 << 20, max_batch_msgs=64)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    torch.cuda.synchronize()
    big = 2 * ((r["nbytes"].astype(np.int64) + 255) // 256 * 256) > (512 << 20)
    assert st["completed"] == (~big).sum() and (res["status"][big] == A.AES_E_BUDGET).all()
    intact = np.nonzero((res["overwritten"] == 0) & (res["status"] == A.AES_OK))[0]
    assert res["overwritten"].sum() > 50 and len(intact) > 20
    o = ref.default()
    for i in intact.tolist():
        n = int(r["nbytes"][i])
        assert oracle_check(o, r[i], keys[i], srv.output(res[i], n)), "request %d (%d bytes)" % (i, n)


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


def test_served_gcm_requests_match_the_oracle(A):
    """GCM requests through the loop (no additional data, the tag after the
    data in the arena): encryptions equal the oracle's ciphertext and tag;
    decryptions of the random payloads equal the oracle's plaintext, and
    both reject the random 'tag' that follows them."""
    r, keys = requests(A, 150, rate=1e5, seed=57, lo=64, hi=1 << 22)
    r["mode"] = A.AES_MODE_GCM
    fp = 2 * ((r["nbytes"].astype(np.int64) + 16 + 255) // 256 * 256)
    cfg = A.serve_cfg(streams=3, budget_bytes=int(fp.sum()) + (1 << 20), max_batch_msgs=32)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    torch.cuda.synchronize()
    assert st["completed"] == len(r) and st["launches"] > 2
    assert (res["status"] == A.AES_OK).all() and not res["overwritten"].any()
    o = ref.default()
    for i, q in enumerate(r):
        n = int(q["nbytes"])
        bits = 128 + 64 * int(q["keybits_code"])
        rk, nr = o.expand_key(keys[i][:bits // 8])
        iv = q["ctr0"][:12]
        payload = seedgen.bytes_np(int(q["payload_seed"]), n)
        got = srv.output(res[i], n).cpu().numpy()
        if q["decrypt"]:
            tag = seedgen.bytes_np(int(q["payload_seed"]), 16, offset=(n + 15) // 16 * 16)
            pt, ok = o.gcm_decrypt(rk, nr, iv, b"", payload, tag)
            assert np.array_equal(got, pt), "request %d plaintext" % i
            assert res["authentic"][i] == int(ok) == 0, "request %d verdict" % i
        else:
            ct, tag = o.gcm_encrypt(rk, nr, iv, b"", payload)
            assert np.array_equal(got, ct), "request %d ciphertext" % i
            assert np.array_equal(srv.tag(res[i], n).cpu().numpy(), tag), "request %d tag" % i
            assert res["authentic"][i] == 1


def test_served_gcm_long_requests(A):
    """Long GCM requests (6 .. 16 MiB, hundreds of MiB per batch, GHASH in
    thousands of pieces): every result equals the single-buffer GCM call on
    the same payload (ciphertext and tag, or plaintext and the refusal of the
    random tag that follows the payload), a separate implementation checked
    against the oracle elsewhere."""
    r, keys = requests(A, 48, rate=1e6, seed=59, lo=6 << 20, hi=16 << 20)
    r["mode"] = A.AES_MODE_GCM
    fp = 2 * ((r["nbytes"].astype(np.int64) + 16 + 255) // 256 * 256)
    cfg = A.serve_cfg(streams=2, budget_bytes=int(fp.sum()) + (1 << 20), max_batch_msgs=64)
    srv = A.Server(keys, cfg)
    res, st = srv.run(r)
    torch.cuda.synchronize()
    assert st["completed"] == len(r)
    assert (res["status"] == A.AES_OK).all() and not res["overwritten"].any()
    ws = torch.empty(A.aes_gcm_workspace_size(), dtype=torch.uint8, device="cuda")
    tag = torch.empty(16, dtype=torch.uint8, device="cuda")
    ok = torch.empty(1, dtype=torch.int32, device="cuda")
    aad = torch.zeros(16, dtype=torch.uint8, device="cuda")
    for i, q in enumerate(r):
        n = int(q["nbytes"])
        pad = (n + 15) // 16 * 16
        bits = 128 + 64 * int(q["keybits_code"])
        rk, nr = A.aes_expand_key(keys[i][:bits // 8])
        iv = q["ctr0"][:12]
        src = seedgen.bytes_torch(int(q["payload_seed"]), pad + 16, "cuda")
        want = torch.empty(n, dtype=torch.uint8, device="cuda")
        got = srv.output(res[i], n)
        if q["decrypt"]:
            A.aes_gcm_decrypt(src[:n], want, n, aad, 0, rk, nr, iv, src[pad:pad + 16], 16, ok, ws)
            torch.cuda.synchronize()
            assert torch.equal(got, want), "request %d plaintext" % i
            assert res["authentic"][i] == int(ok.item()) == 0, "request %d verdict" % i
        else:
            A.aes_gcm_encrypt(src[:n], want, n, aad, 0, rk, nr, iv, tag, ws)
            torch.cuda.synchronize()
            assert torch.equal(got, want), "request %d ciphertext" % i
            assert torch.equal(srv.tag(res[i], n), tag), "request %d tag" % i
            assert res["authentic"][i] == 1
