"""The seeded input streams: host (numpy) and device (torch) versions must
draw the same bytes, since the oracle is fed from the host and the GPU path
from either.  Runs on the CPU (torch's CPU tensors use the same int64 code)."""
import numpy as np
import pytest
import torch

from paper_1611_00463_amd import datagen as G


def test_splitmix_reference_values():
    # SplitMix64 seeded with 0: the first outputs of the published generator
    assert int(G.u64(0, 0)) == 0xE220A8397B1DCDAF
    assert int(G.u64(0, 1)) == 0x6E789E6AA1B965F4


def test_uniform_host_equals_device_stream():
    a = G.uniform_keys(70000, seed=2)
    b = G.uniform_keys_torch(70000, seed=2, device="cpu", chunk=25000).numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dist", G.BALANCE_DISTS)
def test_balance_host_equals_device_stream(dist):
    a = G.balance_keys(dist, 60000, seed=6)
    b = G.balance_keys_torch(dist, 60000, seed=6, device="cpu", chunk=17000).numpy()
    assert np.array_equal(a, b)
    # any slice can be drawn on its own
    assert np.array_equal(G.balance_keys(dist, 1000, seed=6, start=12345), a[12345:13345])


def test_leading_zero_count():
    x = G.u64(9, np.arange(2000, dtype=np.uint64))
    x[:6] = [0, 1, 2, 2 ** 63, 2 ** 62 + 5, 2 ** 64 - 1]
    k = G._clz64(x)
    assert [int(v) for v in k] == [64 - int(v).bit_length() for v in x]


def test_balance_shapes():
    n = 200000
    e = G.balance_keys("exponential", n)
    assert abs(np.mean(e == 0) - 0.5) < 0.01 and abs(np.mean(e == 1) - 0.25) < 0.01
    r = G.balance_keys("right_skewed", n)
    assert r.max() < 65536 and np.median(r) < 65536 / 4  # long right tail
    m = G.balance_keys("normal", n).astype(np.float64)
    # Irwin-Hall of four uniforms on [0, 2^62): mean 2^63, sd 2^62 / sqrt(3)
    assert abs(m.mean() / 2 ** 63 - 1) < 0.01
    assert abs(m.std() / (2 ** 62 / np.sqrt(3)) - 1) < 0.02


@pytest.mark.parametrize("dt", [np.int32, np.int64, np.float32, np.float64])
def test_typed_keys_host_and_device_generators_agree(dt):
    a = G.typed_keys(60000, 7, dt)
    b = G.typed_keys_torch(60000, 7, dt, device="cpu", chunk=25000).numpy()
    assert a.dtype == dt and np.array_equal(a.view(np.uint8), b.view(np.uint8))
    tail = G.typed_keys(30000, 7, dt, start=30000)
    assert np.array_equal(tail.view(np.uint8), a[30000:].view(np.uint8))
    if np.issubdtype(dt, np.floating):
        sp = a[::G.SPECIAL_EVERY]
        assert np.isnan(sp[0]) and np.isnan(sp[1]) and np.signbit(sp[1]) and sp[2] == np.inf and sp[3] == -np.inf
        assert sp[4] == 0 and not np.signbit(sp[4]) and sp[5] == 0 and np.signbit(sp[5])
        fin = np.delete(a, np.arange(0, len(a), G.SPECIAL_EVERY))
        assert np.all(np.abs(fin) <= 2000.0)
