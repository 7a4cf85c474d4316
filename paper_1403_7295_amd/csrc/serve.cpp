// The request loop (aes_serve_run): admission by HBM budget and continuous
// batching over several streams, on one host thread.
//
// Every request owns one arena region (input then output, each rounded up to
// 256 bytes) from admission until its launch has finished; the arena is the
// budget, so admitted bytes never exceed it.  A finished request's output
// stays readable until a later admission is carved from its memory; the loop
// keeps the finished outputs still intact and marks a result overwritten
// when that happens.  Whenever a stream is free,
// everything admitted since the last launch goes out as one batch on it:
// descriptor upload, payload fill, and the batch sequence of
// batch_kernels.hip.  Launches on different streams overlap on the device;
// requests that arrive meanwhile are admitted as memory frees up and ride the
// next free stream.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "aesgpu.h"
#include "arena.h"
#include "internal.h"

namespace aesgpu {
int serve_fail(int status, const std::string &msg);
int serve_device(int *cus, int *batch_grid);
size_t serve_batch_layout(int max_msgs);
int serve_batch_args(const aes_batch *b, BatchKArgs *a);
}  // namespace aesgpu

namespace {

using namespace aesgpu;
using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
constexpr int kMaxStreams = 16;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Per-stream device area: [slot header | descriptors | fill descriptors | batch workspace].
struct SlotHeader {
    int32_t nmsg;
    int32_t pad0;
    uint64_t nchunks;
    uint8_t pad[240];
};
static_assert(sizeof(SlotHeader) == kAlign, "slot header is 256 bytes");

struct ServeLayout {
    size_t arena;
    size_t desc_off, fill_off, ws_off, ws_bytes, slot_bytes, staged_bytes;
    // pinned memory: the staged part, then one reject flag per message, then
    // the GCM fields per message (read and written by the device in place)
    size_t flags_off, gcm_off, host_bytes;
    size_t total;
};

bool make_layout(const aes_serve_cfg &c, ServeLayout *L) {
    if (c.streams < 1 || c.streams > kMaxStreams || c.max_batch_msgs < 1 || c.max_batch_msgs > 65536 ||
        c.budget_bytes < kAlign || c.tile_blocks < 0 || c.tile_blocks > kMaxSplitBlocks ||
        (c.blocks_per_thread != 0 && c.blocks_per_thread != 2 && c.blocks_per_thread != 4))
        return false;
    L->arena = c.budget_bytes / kAlign * kAlign;
    L->desc_off = sizeof(SlotHeader);
    L->fill_off = L->desc_off + round_up(size_t(c.max_batch_msgs) * sizeof(aes_msg_desc), kAlign);
    L->staged_bytes = L->fill_off + round_up(size_t(c.max_batch_msgs) * sizeof(FillDesc), kAlign);
    L->ws_off = L->staged_bytes;
    L->ws_bytes = serve_batch_layout(c.max_batch_msgs);
    L->slot_bytes = L->ws_off + round_up(L->ws_bytes, kAlign);
    L->flags_off = L->staged_bytes;
    L->gcm_off = L->flags_off + round_up(size_t(c.max_batch_msgs), kAlign);
    L->host_bytes = L->gcm_off + round_up(size_t(c.max_batch_msgs) * sizeof(aes_gcm_desc), kAlign);
    L->total = L->arena + size_t(c.streams) * L->slot_bytes;
    return true;
}

struct Slot {
    bool busy = false;
    std::vector<int> reqs;
    double done_at = 0;          // simulated completion time
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr;   // before the descriptor upload
    hipEvent_t ev_fill = nullptr;    // after the payload fill
    hipEvent_t event = nullptr;      // after the batch: the launch is finished
    uint8_t *host = nullptr;     // pinned: staging for header + descriptors, then reject flags
    void *host_dev = nullptr;    // its address on the device
    uint8_t *dev = nullptr;      // this slot's device area
};

struct Loop {
    const aes_request *reqs;
    int nreq;
    const aes_serve_cfg &cfg;
    const ServeLayout &L;
    aes_request_result *res;
    aes_serve_stats st{};
    bool sim;
    int cus = 0;
    int batch_grid = 0;
    const uint8_t *keys;
    int nkeys;
    uint8_t *arena_base;
    std::vector<Slot> slots;
    double device_free_at = 0;   // simulated device
    std::string error;

    Loop(const aes_request *r, int n, const aes_serve_cfg &c, const ServeLayout &l, aes_request_result *o)
        : reqs(r), nreq(n), cfg(c), L(l), res(o), sim(c.simulate_gbps > 0) {}

    // a GCM request's input and output each carry 16 more bytes: the
    // expected tag after the ciphertext (decryption), the tag after the
    // ciphertext (encryption)
    uint64_t payload(int i) const { return reqs[i].nbytes + (reqs[i].mode == AES_MODE_GCM ? 16u : 0u); }
    uint64_t footprint(int i) const { return 2 * round_up(payload(i), kAlign); }

    int launch(Slot &s, double now) {
        const int n = int(s.reqs.size());
        uint64_t bytes = 0;
        for (int i : s.reqs)
            bytes += reqs[i].nbytes;
        if (sim) {
            const double start = std::max(now, device_free_at);
            s.done_at = start + double(bytes) / (cfg.simulate_gbps * 1e9) + 20e-6;
            device_free_at = s.done_at;
            return AES_OK;
        }
        SlotHeader *h = reinterpret_cast<SlotHeader *>(s.host);
        aes_msg_desc *d = reinterpret_cast<aes_msg_desc *>(s.host + L.desc_off);
        FillDesc *f = reinterpret_cast<FillDesc *>(s.host + L.fill_off);
        aes_gcm_desc *g = reinterpret_cast<aes_gcm_desc *>(s.host + L.gcm_off);
        uint64_t chunks = 0;
        // the batch kernel's lists this batch uses; never the fused GCM list:
        // its pieces hold a workgroup for ~0.3 ms each, which lengthened the
        // loop's tail latency without adding measurably to its capacity
        unsigned lists = 0;
        for (int k = 0; k < n; k++) {
            const aes_request &q = reqs[s.reqs[k]];
            const aes_request_result &r = res[s.reqs[k]];
            d[k].in_off = r.in_off;
            d[k].out_off = r.out_off;
            d[k].nbytes = q.nbytes;
            d[k].key_idx = q.key_idx;
            d[k].keybits_code = q.keybits_code;
            d[k].mode = q.mode;
            d[k].decrypt = q.decrypt;
            d[k].reserved = 0;
            std::memcpy(d[k].ctr0, q.ctr0, 16);
            f[k].off = r.in_off;
            f[k].nbytes = payload(s.reqs[k]);
            f[k].seed = q.payload_seed;
            f[k].chunk_first = chunks;
            chunks += (f[k].nbytes + kFillChunk - 1) / kFillChunk;
            const bool inverse = q.decrypt && (q.mode == AES_MODE_ECB || q.mode == AES_MODE_CBC);
            const bool serial = !q.decrypt && q.mode == AES_MODE_CBC;
            lists |= serial ? 4u : inverse ? 2u : 1u;
            if (q.mode == AES_MODE_GCM) {
                // no additional data; the tag 16-byte aligned after the data
                const uint64_t tag_at = (q.nbytes + 15) / 16 * 16;
                g[k].aad_off = r.in_off;
                g[k].aad_bytes = 0;
                g[k].tag_off = (q.decrypt ? r.in_off : r.out_off) + tag_at;
                g[k].tag_bytes = 16;
                g[k].ok = -1;
                lists |= 8u;
            }
        }
        h->nmsg = n;
        h->nchunks = chunks;
        // the prep kernel sets a message's flag if the device-side check
        // refuses it (through the flags' device address)
        std::memset(s.host + L.flags_off, 0, size_t(n));
        // header + descriptors + fill descriptors go up in one copy, made by
        // a kernel on the slot's stream: the next kernels follow it on the
        // same queue, with no hand-off from the copy engine
        const size_t up = round_up(L.fill_off + size_t(n) * sizeof(FillDesc), 16);
        hipError_t e = hipEventRecord(s.ev_start, s.stream);
        if (e == hipSuccess)
            e = launch_stage(s.host_dev, s.dev, up, s.stream);
        FillKArgs fa;
        fa.fd = reinterpret_cast<const FillDesc *>(s.dev + L.fill_off);
        fa.d_nmsg = &reinterpret_cast<const SlotHeader *>(s.dev)->nmsg;
        fa.d_nchunks = &reinterpret_cast<const SlotHeader *>(s.dev)->nchunks;
        fa.base = arena_base;
        if (e == hipSuccess)
            e = launch_fill(fa, std::min<uint64_t>(std::max<uint64_t>(chunks, 1), uint64_t(cus) * 8), s.stream);
        if (e == hipSuccess)
            e = hipEventRecord(s.ev_fill, s.stream);
        if (e == hipSuccess) {
            aes_batch b;
            b.desc = reinterpret_cast<const aes_msg_desc *>(s.dev + L.desc_off);
            b.nmsg = n;
            b.d_nmsg = fa.d_nmsg;
            b.keys = keys;
            b.nkeys = nkeys;
            b.in_base = arena_base;
            b.in_bytes = L.arena;
            b.out_base = arena_base;
            b.out_bytes = L.arena;
            b.workspace = s.dev + L.ws_off;
            b.workspace_bytes = L.ws_bytes;
            b.max_msgs = cfg.max_batch_msgs;
            b.tile_blocks = cfg.tile_blocks;
            b.blocks_per_thread = cfg.blocks_per_thread;
            b.gcm = (lists & 8u) ? reinterpret_cast<aes_gcm_desc *>(static_cast<uint8_t *>(s.host_dev) + L.gcm_off)
                                 : nullptr;
            BatchKArgs ka;
            int st = serve_batch_args(&b, &ka);
            if (st != AES_OK)
                return st;
            ka.reject_flags = static_cast<uint8_t *>(s.host_dev) + L.flags_off;
            e = launch_batch(ka, batch_grid, s.stream, lists, n);
        }
        if (e == hipSuccess)
            e = hipEventRecord(s.event, s.stream);
        if (e != hipSuccess) {
            error = std::string("launch: ") + hipGetErrorString(e);
            return AES_E_DEVICE;
        }
        return AES_OK;
    }

    // 1 = finished, 0 = still running, <0 = error
    int finished(Slot &s, double now) {
        if (sim)
            return now >= s.done_at ? 1 : 0;
        hipError_t e = hipEventQuery(s.event);
        if (e == hipSuccess) {
            // device time of the payload fill (with the descriptor upload)
            // and of the batch, per launch (launches on other streams may
            // share the device meanwhile)
            float fill_ms = 0, cipher_ms = 0;
            if (hipEventElapsedTime(&fill_ms, s.ev_start, s.ev_fill) == hipSuccess &&
                hipEventElapsedTime(&cipher_ms, s.ev_fill, s.event) == hipSuccess) {
                st.fill_device_s += 1e-3 * fill_ms;
                st.cipher_device_s += 1e-3 * cipher_ms;
            }
            return 1;
        }
        if (e == hipErrorNotReady)
            return 0;
        error = std::string("event query: ") + hipGetErrorString(e);
        return -1;
    }

    // Outputs of finished requests that no later admission has touched yet,
    // by start offset: [start, end) and the request.  They never overlap each
    // other (an admission removes every one it overlaps before its own
    // output can join).
    struct Region {
        uint64_t end;
        int req;
    };
    std::map<uint64_t, Region> intact;

    void mark_overwritten(uint64_t lo, uint64_t hi) {
        auto it = intact.upper_bound(lo);
        if (it != intact.begin() && std::prev(it)->second.end > lo)
            --it;
        while (it != intact.end() && it->first < hi) {
            res[it->second.req].overwritten = 1;
            it = intact.erase(it);
        }
    }

    int run() {
        Arena arena(L.arena);
        std::deque<int> queue;     // arrived, waiting for budget
        std::vector<int> pending;  // admitted, waiting for a stream
        int next = 0, settled = 0, inflight = 0, launches = 0;
        uint64_t inflight_bytes = 0;
        double first_arrival = nreq ? reqs[0].arrival_s : 0, last_done = first_arrival;
        const double timeout = cfg.timeout_s > 0 ? cfg.timeout_s : 60.0;
        const auto t0 = Clock::now();
        double last_progress = 0;
        auto clock = [&] { return std::chrono::duration<double>(Clock::now() - t0).count(); };

        while (settled < nreq) {
            double now = clock();
            bool progress = false;
            // 1. launches that have finished
            for (Slot &s : slots) {
                if (!s.busy)
                    continue;
                const int f = finished(s, now);
                if (f < 0)
                    return AES_E_DEVICE;
                if (f == 0)
                    continue;
                const double t = sim ? s.done_at : now;
                const uint8_t *flags = sim ? nullptr : s.host + L.flags_off;
                const aes_gcm_desc *g = sim ? nullptr : reinterpret_cast<const aes_gcm_desc *>(s.host + L.gcm_off);
                for (size_t k = 0; k < s.reqs.size(); k++) {
                    const int i = s.reqs[k];
                    res[i].latency_s = t - reqs[i].arrival_s;
                    res[i].status = flags && flags[k] ? AES_E_ARG : AES_OK;
                    if (reqs[i].mode == AES_MODE_GCM)
                        res[i].authentic = g ? g[k].ok : (reqs[i].decrypt ? 0 : 1);
                    const uint64_t fp = footprint(i);
                    if (fp) {
                        arena.release(res[i].in_off, fp);
                        if (res[i].status == AES_OK)
                            intact[res[i].out_off] = Region{res[i].out_off + fp / 2, i};
                    }
                    inflight_bytes -= fp;
                    inflight--;
                    st.bytes_done += reqs[i].nbytes;
                    st.completed++;
                    settled++;
                }
                last_done = std::max(last_done, t);
                s.reqs.clear();
                s.busy = false;
                progress = true;
            }
            // 2. arrivals
            while (next < nreq && reqs[next].arrival_s <= now) {
                queue.push_back(next++);
                progress = true;
            }
            // 3. admission, in arrival order, while the budget has room
            while (!queue.empty() && int(pending.size()) < cfg.max_batch_msgs) {
                const int i = queue.front();
                const uint64_t fp = footprint(i);
                if (fp > L.arena) {
                    res[i].status = AES_E_BUDGET;
                    res[i].latency_s = -1;
                    st.rejected++;
                    settled++;
                    queue.pop_front();
                    progress = true;
                    continue;
                }
                uint64_t off = 0;
                if (fp && !arena.alloc(fp, &off))
                    break;
                if (fp)
                    mark_overwritten(off, off + fp);
                res[i].in_off = off;
                res[i].out_off = off + fp / 2;
                res[i].admit_s = now - reqs[i].arrival_s;
                inflight++;
                inflight_bytes += fp;
                st.max_inflight_reqs = std::max(st.max_inflight_reqs, inflight);
                st.max_inflight_bytes = std::max(st.max_inflight_bytes, inflight_bytes);
                pending.push_back(i);
                queue.pop_front();
                progress = true;
            }
            // 4. launch what is admitted on a free stream
            if (!pending.empty()) {
                for (Slot &s : slots) {
                    if (s.busy)
                        continue;
                    s.reqs.swap(pending);
                    pending.clear();
                    for (int i : s.reqs)
                        res[i].launch = launches;
                    const int rc = launch(s, now);
                    if (rc != AES_OK)
                        return rc;
                    s.busy = true;
                    launches++;
                    progress = true;
                    break;
                }
            }
            if (progress) {
                last_progress = now;
                continue;
            }
            bool busy = false;
            for (Slot &s : slots)
                busy |= s.busy;
            if (busy && now - last_progress > timeout) {
                error = "no launch finished within the timeout";
                return AES_E_DEVICE;
            }
            std::this_thread::yield();
        }
        st.span_s = last_done - first_arrival;
        st.launches = launches;
        return AES_OK;
    }
};

}  // namespace

extern "C" {

int aes_serve_scratch_size(const aes_serve_cfg *cfg, size_t *bytes) {
    if (!cfg || !bytes)
        return serve_fail(AES_E_NULL, "cfg and bytes must not be NULL");
    ServeLayout L;
    if (!make_layout(*cfg, &L))
        return serve_fail(AES_E_ARG, "streams 1..16, max_batch_msgs 1..65536, budget_bytes >= 256, "
                                     "tile_blocks 0 .. 1024, blocks_per_thread 0, 2 or 4");
    *bytes = L.total;
    return AES_OK;
}

int aes_serve_run(const aes_request *reqs, int nreq, const uint8_t *d_keys, int nkeys, void *d_scratch,
                  size_t scratch_bytes, const aes_serve_cfg *cfg, aes_request_result *results,
                  aes_serve_stats *stats) {
    if (!cfg || (!reqs && nreq > 0) || (!results && nreq > 0))
        return serve_fail(AES_E_NULL, "cfg, reqs and results must not be NULL");
    ServeLayout L;
    if (!make_layout(*cfg, &L))
        return serve_fail(AES_E_ARG, "bad serve configuration");
    if (nreq < 0)
        return serve_fail(AES_E_ARG, "nreq must be >= 0");
    if (nkeys < 1)
        return serve_fail(AES_E_ARG, "nkeys must be >= 1");
    for (int i = 0; i < nreq; i++) {
        const aes_request &q = reqs[i];
        if (i && q.arrival_s < reqs[i - 1].arrival_s)
            return serve_fail(AES_E_ARG, "requests must be sorted by arrival_s");
        if (q.keybits_code > 2 || (q.mode > AES_MODE_CBC && q.mode != AES_MODE_GCM) || q.decrypt > 1 ||
            q.key_idx >= uint32_t(nkeys))
            return serve_fail(AES_E_ARG, "request " + std::to_string(i) + ": bad key, mode or direction");
        if (q.mode == AES_MODE_GCM && q.nbytes > (uint64_t(1) << 36) - 32)
            return serve_fail(AES_E_LENGTH, "request " + std::to_string(i) + ": GCM longer than 2^36 - 32 bytes");
        if ((q.mode == AES_MODE_ECB || q.mode == AES_MODE_CBC) && q.nbytes % 16)
            return serve_fail(AES_E_LENGTH, "request " + std::to_string(i) + ": ECB/CBC length not whole blocks");
        if (q.mode == AES_MODE_CTR && q.nbytes > kCtrMaxBytes)
            return serve_fail(AES_E_LENGTH, "request " + std::to_string(i) + ": CTR longer than 2^36 bytes");
    }
    const bool sim = cfg->simulate_gbps > 0;
    Loop loop(reqs, nreq, *cfg, L, results);
    for (int i = 0; i < nreq; i++) {
        results[i] = aes_request_result{};
        results[i].status = AES_E_ARG;
        results[i].launch = -1;
        results[i].authentic = -1;
    }
    loop.keys = d_keys;
    loop.nkeys = nkeys;
    loop.slots.resize(cfg->streams);
    int rc = AES_OK;
    if (!sim) {
        if (!d_keys || !d_scratch)
            return serve_fail(AES_E_NULL, "d_keys and d_scratch must not be NULL");
        if (reinterpret_cast<uintptr_t>(d_scratch) & (kAlign - 1))
            return serve_fail(AES_E_ALIGN, "d_scratch must be 256-byte aligned");
        if (scratch_bytes < L.total)
            return serve_fail(AES_E_LENGTH, "scratch smaller than aes_serve_scratch_size reports");
        rc = serve_device(&loop.cus, &loop.batch_grid);
        if (rc != AES_OK)
            return rc;
        loop.arena_base = static_cast<uint8_t *>(d_scratch);
        hipError_t e = hipSuccess;
        for (int k = 0; k < cfg->streams && e == hipSuccess; k++) {
            Slot &s = loop.slots[k];
            s.dev = loop.arena_base + L.arena + size_t(k) * L.slot_bytes;
            e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipEventCreate(&s.ev_start);
            if (e == hipSuccess)
                e = hipEventCreate(&s.ev_fill);
            if (e == hipSuccess)
                e = hipEventCreate(&s.event);
            if (e == hipSuccess)
                e = hipHostMalloc(reinterpret_cast<void **>(&s.host), L.host_bytes, hipHostMallocDefault);
            if (e == hipSuccess)
                e = hipHostGetDevicePointer(&s.host_dev, s.host, 0);
        }
        if (e != hipSuccess) {
            loop.error = std::string("stream set-up: ") + hipGetErrorString(e);
            rc = AES_E_DEVICE;
        }
    }
    if (rc == AES_OK)
        rc = loop.run();
    if (!sim) {
        // drain whatever is still in flight before the staging memory goes away
        for (Slot &s : loop.slots)
            if (s.stream)
                (void)hipStreamSynchronize(s.stream);
        for (Slot &s : loop.slots) {
            if (s.host)
                (void)hipHostFree(s.host);
            if (s.event)
                (void)hipEventDestroy(s.event);
            if (s.ev_fill)
                (void)hipEventDestroy(s.ev_fill);
            if (s.ev_start)
                (void)hipEventDestroy(s.ev_start);
            if (s.stream)
                (void)hipStreamDestroy(s.stream);
        }
    }
    if (stats)
        *stats = loop.st;
    if (rc != AES_OK)
        return serve_fail(rc, loop.error.empty() ? "serve loop failed" : loop.error);
    return AES_OK;
}

}  // extern "C"
