"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  It holds no AES arithmetic, only a counter-based pseudo-random
generator, so that both sides of every parity check read the same bytes.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used in counter form.  Word i of the stream
with seed s is

    mix64(s + (i + 1) * 0x9E3779B97F4A7C15  mod 2^64)

where mix64 is SplitMix64's published output function.  A byte stream is the
words in order, each stored little-endian, so byte b of the stream is byte
b mod 8 of word b // 8.  Because word i depends only on (s, i), any slice of
a stream can be produced on its own; that is what lets tests check a sample
of a 1 GiB output without producing the whole input on the host.

Stream seeds are derived from a master seed, a tag and an index:
    stream_seed(master, tag, index) = mix64(master ^ (tag << 56) ^ index)
with tags DATA = 1, KEY = 2, NONCE = 3, LEN = 4.

Two implementations of the same definition live here: numpy (host) and
torch (any device, used to fill large device buffers without a host copy).
A test checks that they agree.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

TAG_DATA, TAG_KEY, TAG_NONCE, TAG_LEN = 1, 2, 3, 4


def mix64(z):
    """SplitMix64's output function on one Python int."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def stream_seed(master, tag, index=0):
    return mix64((master ^ (tag << 56) ^ index) & MASK64)


def words_np(seed, first, count):
    """Words first .. first+count-1 of stream `seed`, as numpy uint64."""
    i = np.arange(first + 1, first + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        z = z ^ (z >> np.uint64(31))
    return z


def bytes_np(seed, nbytes, offset=0):
    """Bytes offset .. offset+nbytes-1 of stream `seed`, as numpy uint8."""
    if nbytes == 0:
        return np.zeros(0, np.uint8)
    w0 = offset // 8
    w1 = (offset + nbytes + 7) // 8
    raw = words_np(seed, w0, w1 - w0).astype("<u8").view(np.uint8)
    start = offset - 8 * w0
    return raw[start:start + nbytes].copy()


def _signed(c):
    return c - (1 << 64) if c >= (1 << 63) else c


def _srl(torch, z, s):
    # logical right shift of int64 values read as unsigned 64-bit words
    return (z >> s) & ((1 << (64 - s)) - 1)


def bytes_torch(seed, nbytes, device, chunk_words=1 << 26):
    """The first nbytes of stream `seed` as a torch uint8 tensor on `device`.

    int64 arithmetic in torch wraps modulo 2^64, which is the unsigned
    arithmetic of the definition read in two's complement.
    """
    import torch
    nwords = (nbytes + 7) // 8
    out = torch.empty(nwords * 8, dtype=torch.uint8, device=device)
    outw = out.view(torch.int64)
    s = _signed(seed & MASK64)
    g, m1, m2 = _signed(GAMMA), _signed(MIX1), _signed(MIX2)
    for w0 in range(0, nwords, chunk_words):
        n = min(chunk_words, nwords - w0)
        z = torch.arange(w0 + 1, w0 + 1 + n, dtype=torch.int64, device=device)
        z.mul_(g).add_(s)
        z = (z ^ _srl(torch, z, 30)).mul_(m1)
        z = (z ^ _srl(torch, z, 27)).mul_(m2)
        z = z ^ _srl(torch, z, 31)
        outw[w0:w0 + n] = z
        del z
    return out[:nbytes]


def data_np(master, index, nbytes, offset=0):
    return bytes_np(stream_seed(master, TAG_DATA, index), nbytes, offset)


def data_torch(master, index, nbytes, device):
    return bytes_torch(stream_seed(master, TAG_DATA, index), nbytes, device)


def key(master, index, keybits):
    return bytes_np(stream_seed(master, TAG_KEY, index), keybits // 8)


def nonce(master, index):
    """A 16-byte initial counter block: 12 random nonce bytes, counter 0."""
    n = bytes_np(stream_seed(master, TAG_NONCE, index), 12)
    return np.concatenate([n, np.zeros(4, np.uint8)])


# --- workload shapes -------------------------------------------------------
def log_uniform_lengths(rng, n, lo, hi, multiple=1):
    """n lengths with log2(length) uniform between log2(lo) and log2(hi),
    rounded to the nearest multiple of `multiple` (at least `multiple`)."""
    u = rng.random(n)
    raw = lo * (hi / lo) ** u
    out = np.maximum(np.rint(raw / multiple), 1).astype(np.int64) * multiple
    return np.minimum(out, hi)


def ragged_batch(master, n, lo=16, hi=1 << 24, multiple=16):
    """The ragged multi-message workload: n messages with lengths
    log-uniform in [lo, hi] (multiples of 16 by default), AES-128 or AES-256
    with probability 1/2 each.  Returns (lengths, keybits, keys[n, 32],
    nonces[n, 16]); key and nonce m come from the KEY / NONCE streams with
    index m."""
    rng = np.random.default_rng(master)
    lengths = log_uniform_lengths(rng, n, lo, hi, multiple)
    keybits = np.where(rng.random(n) < 0.5, 128, 256)
    keys = np.zeros((n, 32), np.uint8)
    nonces = np.zeros((n, 16), np.uint8)
    for m in range(n):
        keys[m, :keybits[m] // 8] = key(master, m, int(keybits[m]))
        nonces[m] = nonce(master, m)
    return lengths, keybits, keys, nonces


def served_requests(master, n, rate, lo=64, hi=1 << 26, enc_fraction=0.7, start=0.0):
    """The served workload: n requests with Poisson arrivals at `rate` per
    second, sizes log-uniform in [lo, hi] bytes (byte-granular), encrypt with
    probability enc_fraction else decrypt, AES-128 or AES-256 (1/2 each), all
    CTR, each with its own key slot, nonce and payload stream.  Returns
    (fields dict of numpy arrays, keys[n, 32]); request m uses key slot m,
    nonce m and payload seed stream_seed(master, DATA, m)."""
    rng = np.random.default_rng(master)
    gaps = rng.exponential(1.0 / rate, n)
    arrival = start + np.cumsum(gaps) - gaps[0]
    nbytes = log_uniform_lengths(rng, n, lo, hi, 1)
    decrypt = (rng.random(n) >= enc_fraction).astype(np.uint8)
    keybits = np.where(rng.random(n) < 0.5, 128, 256)
    keys = np.zeros((n, 32), np.uint8)
    ctr0 = np.zeros((n, 16), np.uint8)
    seeds = np.zeros(n, np.uint64)
    for m in range(n):
        keys[m, :keybits[m] // 8] = key(master, m, int(keybits[m]))
        ctr0[m] = nonce(master, m)
        seeds[m] = stream_seed(master, TAG_DATA, m)
    return {"arrival_s": arrival, "nbytes": nbytes, "payload_seed": seeds, "key_idx": np.arange(n),
            "keybits_code": (keybits - 128) // 64, "mode": np.ones(n, np.uint8),
            "decrypt": decrypt, "ctr0": ctr0}, keys
