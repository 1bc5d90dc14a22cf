"""Pins of the oracle's coder and of whole-pipeline round trips.

The coder is pinned by brute force (every short sequence over small
alphabets) and by code length against the ideal -log2 of the coded
probabilities; the pipeline by exact round trips, by the order independence
of the decoded image (Sec. 3: parallel decoding does not change the result)
and by NaN poisoning of pixels that a schedule has not produced yet.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth


def row_from_freqs(f):
    return np.concatenate([[0], np.cumsum(f)]).astype(np.int32)


def small_rows():
    """CDF rows over 3 live symbols padded to 256 with 1-count symbols."""
    rows = []
    for a, b in [(1, 1), (30000, 200), (65000, 10), (100, 100), (21760, 21760)]:
        f = np.ones(256, dtype=np.int64)
        f[0], f[1] = a, b
        f[2] = 65536 - f.sum() + f[2]
        assert f[2] >= 1 and f.sum() == 65536
        rows.append(row_from_freqs(f))
    return rows


def test_rans_bruteforce_short_sequences():
    rows = small_rows()
    for n in range(1, 5):
        for syms in itertools.product(range(3), repeat=n):
            for rsel in itertools.product(range(len(rows)), repeat=min(n, 2)):
                cd = np.stack([rows[rsel[k % len(rsel)]] for k in range(n)])
                st = [cd[k, s] for k, s in enumerate(syms)]
                fr = [cd[k, s + 1] - cd[k, s] for k, s in enumerate(syms)]
                data = oracle.rans_encode(st, fr)
                dec, ok = oracle.rans_decode(cd, data)
                assert ok and list(dec) == list(syms)
                ideal = -sum(math.log2(f / 65536) for f in fr)
                assert len(data) * 8 <= ideal + 32 + 1e-9


def random_rows(rng, N, peak):
    w = rng.random((N, 256)) ** peak + 1e-4
    w /= w.sum(1, keepdims=True)
    f = 1 + np.floor(w * 65280).astype(np.int64)
    f[np.arange(N), np.argmax(f, 1)] += 65536 - f.sum(1)
    return np.concatenate([np.zeros((N, 1), np.int64), np.cumsum(f, 1)], 1).astype(np.int32), f


@pytest.mark.parametrize("seed,N,peak", [(0, 1, 1), (1, 50, 2), (2, 3072, 8), (3, 20000, 30), (4, 12288, 1)])
def test_rans_random_sequences(seed, N, peak):
    rng = np.random.default_rng(seed)
    cd, f = random_rows(rng, N, peak)
    syms = np.array([rng.choice(256, p=f[n] / 65536.0) for n in range(N)])
    st = cd[np.arange(N), syms]
    fr = cd[np.arange(N), syms + 1] - st
    data = oracle.rans_encode(st, fr)
    dec, ok = oracle.rans_decode(cd, data)
    assert ok and (dec == syms).all()
    ideal = float(-np.log2(fr / 65536.0).sum())
    assert len(data) * 8 <= ideal + 32
    # flipping any single byte must not decode cleanly to the same symbols
    for k in rng.choice(len(data), size=min(len(data), 20), replace=False):
        bad = bytearray(data)
        bad[k] ^= 0x5A
        d2, ok2 = oracle.rans_decode(cd, bytes(bad))
        assert not (ok2 and (d2 == syms).all())


def test_rans_truncated_stream_rejected():
    rng = np.random.default_rng(9)
    cd, f = random_rows(rng, 500, 3)
    syms = np.array([rng.choice(256, p=f[n] / 65536.0) for n in range(500)])
    st = cd[np.arange(500), syms]
    data = oracle.rans_encode(st, cd[np.arange(500), syms + 1] - st)
    for cut in (0, 1, 3, len(data) - 1):
        _, ok = oracle.rans_decode(cd, data[:cut])
        assert not ok


@pytest.fixture(scope="module")
def tiny_model():
    d = synth.MODEL_DIMS["tiny"]
    p = synth.init_params(d["h"], d["C"], d["n_blocks"], d["seed"]).astype(np.float64)
    return oracle.Model.from_params(d["h"], d["C"], d["n_blocks"], p)


def test_pipeline_1x1_all_values(tiny_model):
    for v in range(256):
        img = np.array([[[v, (7 * v) % 256, (13 * v + 5) % 256]]], dtype=np.uint8)
        for order in (0, 1):
            data = tiny_model.encode(img, order)
            assert np.array_equal(tiny_model.decode(data, 1, 1, order), img)


@pytest.mark.parametrize("H,W", [(1, 2), (2, 1), (2, 2), (3, 5), (5, 3), (4, 9), (9, 4)])
def test_pipeline_tiny_random(tiny_model, H, W):
    rng = np.random.default_rng(H * 100 + W)
    for _ in range(3):
        img = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
        for order in (0, 1):
            for ph, pw in [(0, 0), (2, 2), (1, 3)]:
                data = tiny_model.encode(img, order, ph, pw)
                assert np.array_equal(tiny_model.decode(data, H, W, order, ph, pw), img)


def test_order_independence_and_poisoning():
    blob, _ = synth.model_blob("A")
    m = oracle.Model.from_blob(blob)
    img = synth.smooth_field_image(2.0, 3, 0, 12, 14, 77)
    raster = m.encode(img, 0)
    wave = m.encode(img, 1)
    # both decodes run on a NaN-poisoned canvas; the wavefront one reads a
    # poisoned pixel if its schedule were not causal
    assert np.array_equal(m.decode(raster, 12, 14, 0), img)
    assert np.array_equal(m.decode(wave, 12, 14, 1), img)
    # same CDFs, so the same ideal code length; stream lengths agree to within
    # the coder's few bytes of start-up and flush
    assert abs(len(raster) - len(wave)) <= 4
    # an offset larger than h+1 is also causal
    assert np.array_equal(m.decode(m.encode(img, 1, offset=m.h + 2), 12, 14, 1, offset=m.h + 2), img)
    # step j + h*i is not: the poisoned canvas reaches the model
    with pytest.raises(oracle.OracleError) as e:
        m.decode(m.encode(img, 1, offset=m.h), 12, 14, 1, offset=m.h)
    assert e.value.code == oracle.E_NAN


def test_corrupt_container_rejected(tiny_model):
    img = synth.smooth_field_image(2.0, 3, 0, 6, 6, 3)
    data = bytearray(tiny_model.encode(img, 1))
    bad = bytearray(data)
    bad[-1] ^= 0xFF
    with pytest.raises(oracle.OracleError):
        tiny_model.decode(bytes(bad), 6, 6, 1)
    with pytest.raises(oracle.OracleError):
        tiny_model.decode(bytes(data[:-1]), 6, 6, 1)


@pytest.mark.parametrize("ph,pw", [(32, 32), (64, 64), (16, 24), (7, 5)])
def test_patch_equals_per_crop(ph, pw):
    blob, _ = synth.model_blob("tiny")
    m = oracle.Model.from_blob(blob)
    img = synth.smooth_field_image(2.0, 3, 0, 40, 50, 5)
    H, W, _ = img.shape
    s = m.stats(img, ph, pw)
    q = c = 0.0
    for y in range(0, H, ph):
        for x in range(0, W, pw):
            r = m.stats(img[y:y + ph, x:x + pw].copy())
            q += r["qbits"]
            c += r["cbits"]
    assert abs(s["qbits"] - q) <= 1e-9 * q and abs(s["cbits"] - c) <= 1e-9 * c
    # a patch covering the whole image is the unpatched method
    full = m.stats(img)
    big = m.stats(img, 4 * H, 4 * W)
    assert full == big
    data = m.encode(img, 1, ph, pw)
    assert np.array_equal(m.decode(data, H, W, 1, ph, pw), img)
