"""The shared input generator: its numpy and torch forms agree with the
scalar definition, and slices are consistent with the whole stream."""
import numpy as np

import seedgen


def test_numpy_matches_scalar_definition():
    seed = seedgen.stream_seed(3, seedgen.TAG_DATA, 5)
    w = seedgen.words_np(seed, 0, 64)
    for i in range(64):
        z = (seed + (i + 1) * seedgen.GAMMA) & seedgen.MASK64
        assert int(w[i]) == seedgen.mix64(z)


def test_slices_agree_with_whole_stream():
    seed = 0x1234
    whole = seedgen.bytes_np(seed, 1000)
    for off, n in ((0, 1), (3, 17), (8, 64), (999, 1), (5, 995)):
        assert np.array_equal(seedgen.bytes_np(seed, n, off), whole[off:off + n])


def test_torch_cpu_matches_numpy():
    import torch
    seed = seedgen.stream_seed(9, seedgen.TAG_DATA, 0)
    for n in (0, 1, 7, 8, 4096 + 5):
        t = seedgen.bytes_torch(seed, n, "cpu", chunk_words=100).numpy()
        assert np.array_equal(t, seedgen.bytes_np(seed, n)), n
    assert torch.uint8 == seedgen.bytes_torch(seed, 3, "cpu").dtype


def test_keys_and_nonces():
    assert seedgen.key(1, 0, 128).size == 16
    assert seedgen.key(1, 0, 256).size == 32
    n = seedgen.nonce(1, 0)
    assert n.size == 16 and not n[12:].any()
    assert not np.array_equal(seedgen.key(1, 0, 128), seedgen.key(1, 1, 128))
