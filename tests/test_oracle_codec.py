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
    """Every sequence of up to four symbols over three live symbols, with
    several CDF rows, round-trips. Code length bound: each push adds at most
    log2(M/f) + 1 bits to log2(x + 1) (a spread push lands below
    (x + 1) 2^(16-p) <= (x + 1) 2M/f; a range push from x >= f below
    (M/f)(x + f) < (M/f) 2 (x + 1)), emissions happen only above 2^15 and
    add under 0.012 bits each, the start state 1 is log2(2) = 1 bit, and the
    flush rounds log2(x + 1) up to whole bytes: len <= ideal + n + 9 bits
    (+ emissions, none this short)."""
    rows = small_rows()
    for n in range(0, 5):
        for syms in itertools.product(range(3), repeat=n):
            for rsel in itertools.product(range(len(rows)), repeat=min(n, 2)):
                cd = np.stack([rows[rsel[k % len(rsel)]] for k in range(n)]) if n else np.zeros((0, 257), np.int32)
                st = [cd[k, s] for k, s in enumerate(syms)]
                fr = [cd[k, s + 1] - cd[k, s] for k, s in enumerate(syms)]
                data = oracle.rans_encode(st, fr)
                dec, ok = oracle.rans_decode(cd, data)
                assert ok and list(dec) == list(syms)
                ideal = -sum(math.log2(f / 65536) for f in fr)
                assert len(data) * 8 <= ideal + n + 9 + 1e-9


def rev16(v):
    return int(format(v, "016b")[::-1], 2)


def test_spread_slots_worked_example():
    """Symbol range [8, 13): 8 = 1000b, 9 = 1001b, 10 = 1010b, 11 = 1011b,
    12 = 1100b reverse (16 bits) to 0x1000, 0x9000, 0x5000, 0xD000, 0x3000;
    in increasing order these are the slots of pushes from x = 0..4."""
    want = [0x1000, 0x3000, 0x5000, 0x9000, 0xD000]
    assert [oracle.spread_select(x, 8, 5) for x in range(5)] == want
    assert [oracle.spread_rank(y, 8, 5) for y in want] == list(range(5))
    assert oracle.spread_select(5, 8, 5) == 65536  # no sixth slot
    # start 0: slot 0 reverses to 0, so a zero state stays zero; the next
    # slot below 300 is 2 (0x4000 reversed is 2, 0x8000 is 1)
    assert oracle.spread_select(0, 0, 300) == 0
    assert oracle.spread_select(1, 0, 300) == 0x80 and oracle.spread_select(1, 0, 20000) == 2


@pytest.mark.parametrize("seed", range(6))
def test_spread_slots_bound_and_inverse(seed):
    """For random ranges [s, s + f): the slots are increasing in x, each
    reverses into the range, rank inverts select, and slot x lies below
    (x + 1) 2^(16-p) with 2^p <= f (the range holds every residue modulo 2^p,
    so every block of 2^(16-p) slots holds one)."""
    rng = np.random.default_rng(seed)
    for _ in range(4):
        f = int(rng.integers(1, 65536 - 255)) if seed % 2 else int(rng.integers(1, 40))
        s = int(rng.integers(0, 65536 - f + 1))
        p = f.bit_length() - 1
        xs = sorted(set(x for x in [0, 1, f - 1] + list(rng.integers(0, f, size=20)) if x < f))
        ys = [oracle.spread_select(x, s, f) for x in xs]
        assert all(a < b for a, b in zip(ys, ys[1:]))
        for x, y in zip(xs, ys):
            assert s <= rev16(y) < s + f
            assert oracle.spread_rank(y, s, f) == x
            assert y < (x + 1) << (16 - p)


def test_spread_slots_partition_a_row():
    """The spread slots of the 256 symbols of a CDF row cover [0, 2^16)
    exactly once: counted by rank at 2^16 they sum to 2^16, and every slot
    belongs to the symbol its reversal falls in."""
    rng = np.random.default_rng(5)
    cd, f = random_rows(rng, 1, 2)
    row = cd[0]
    tot = sum(oracle.spread_rank(65536, int(row[k]), int(row[k + 1] - row[k])) for k in range(256))
    assert tot == 65536
    for y in rng.integers(0, 65536, size=50):
        k = int(np.searchsorted(row, rev16(int(y)), side="right") - 1)
        x = oracle.spread_rank(int(y), int(row[k]), int(row[k + 1] - row[k]))
        assert oracle.spread_select(x, int(row[k]), int(row[k + 1] - row[k])) == y


def random_rows(rng, N, peak):
    w = rng.random((N, 256)) ** peak + 1e-4
    w /= w.sum(1, keepdims=True)
    f = 1 + np.floor(w * 65280).astype(np.int64)
    f[np.arange(N), np.argmax(f, 1)] += 65536 - f.sum(1)
    return np.concatenate([np.zeros((N, 1), np.int64), np.cumsum(f, 1)], 1).astype(np.int32), f


@pytest.mark.parametrize("seed,N,peak", [(0, 1, 1), (1, 50, 2), (2, 3072, 8), (3, 20000, 30), (4, 12288, 1)])
def test_rans_random_sequences(seed, N, peak):
    """Random rows and symbols drawn from them round-trip. Code length: once
    the state is at least 2^7 f a push adds at most log2(M/f) + log2(1 +
    2^-7) bits, an emission at most 0.012; the start (states below that) is
    allowed 16 bits and the flush rounding 8."""
    rng = np.random.default_rng(seed)
    cd, f = random_rows(rng, N, peak)
    syms = np.array([rng.choice(256, p=f[n] / 65536.0) for n in range(N)])
    st = cd[np.arange(N), syms]
    fr = cd[np.arange(N), syms + 1] - st
    data = oracle.rans_encode(st, fr)
    dec, ok = oracle.rans_decode(cd, data)
    assert ok and (dec == syms).all()
    ideal = float(-np.log2(fr / 65536.0).sum())
    assert len(data) * 8 <= ideal + 16 + 8 + 0.0113 * (N + len(data))
    # flipping any single byte must not decode cleanly to the same symbols
    for k in rng.choice(len(data), size=min(len(data), 20), replace=False):
        bad = bytearray(data)
        bad[k] ^= 0x5A
        d2, ok2 = oracle.rans_decode(cd, bytes(bad))
        assert not (ok2 and (d2 == syms).all())


def test_rans_overhead_per_stream():
    """The point of the start and flush rules: over many streams at 2..9 bits
    per symbol, the coded length exceeds the ideal -log2 of the coded
    probabilities by about the rounding of the last byte (mean below 5 bits,
    none above 16). A coder that starts from a fixed state (x0 = 1, where the
    first pushes jump to the symbol's range start) and flushes four bytes
    costs 12-16 bits per stream here."""
    rng = np.random.default_rng(21)
    over = []
    for t in range(120):
        N = int(rng.integers(30, 1500))
        cd, f = random_rows(rng, 8, float(rng.choice([1, 4, 16, 40])))
        rsel = rng.integers(0, 8, size=N)
        syms = np.array([rng.choice(256, p=f[r] / 65536.0) for r in rsel])
        st = cd[rsel, syms]
        fr = cd[rsel, syms + 1] - st
        data = oracle.rans_encode(st, fr)
        dec, ok = oracle.rans_decode(cd[rsel], data)
        assert ok and (dec == syms).all()
        over.append(len(data) * 8 + float(np.log2(fr / 65536.0).sum()))
    over = np.array(over)
    assert over.mean() < 5.0 and over.max() < 16.0, (over.mean(), over.max())


def test_rans_truncated_stream_rejected():
    """A stream cut short is rejected: its decoder runs out of bytes early,
    its state drains to 0 (a spread pop maps a state below 2^16 to at most
    itself, and 0 to 0) and cannot end in the start state 1."""
    rng = np.random.default_rng(9)
    cd, f = random_rows(rng, 500, 3)
    syms = np.array([rng.choice(256, p=f[n] / 65536.0) for n in range(500)])
    st = cd[np.arange(500), syms]
    data = oracle.rans_encode(st, cd[np.arange(500), syms + 1] - st)
    for cut in (0, 1, 3, len(data) - 2, len(data) - 1):
        _, ok = oracle.rans_decode(cd, data[:cut])
        assert not ok


def test_rans_empty_stream():
    """No symbols: the start state alone, one byte."""
    assert oracle.rans_encode([], []) == b"\x01"
    assert oracle.rans_decode(np.zeros((0, 257), np.int32), b"\x01")[1]
    assert not oracle.rans_decode(np.zeros((0, 257), np.int32), b"")[1]


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
    assert abs(len(raster) - len(wave)) <= 3
    # an offset larger than h+1 is also causal
    assert np.array_equal(m.decode(m.encode(img, 1, offset=m.h + 2), 12, 14, 1, offset=m.h + 2), img)
    # step j + h*i is not: the poisoned canvas reaches the model
    with pytest.raises(oracle.OracleError) as e:
        m.decode(m.encode(img, 1, offset=m.h), 12, 14, 1, offset=m.h)
    assert e.value.code == oracle.E_NAN


def test_corrupt_container_rejected(tiny_model):
    """A container cut by one byte is rejected (its last stream drains to 0);
    so is one with a damaged byte in the middle of its stream. (The coder's
    only redundancy is its start state, about one bit: a damaged last byte
    changes only the last few, contracted, spread pops and can end in the
    start state by chance; the GPU container adds an image checksum.)"""
    img = synth.smooth_field_image(2.0, 3, 0, 6, 6, 3)
    data = bytearray(tiny_model.encode(img, 1))
    bad = bytearray(data)
    bad[len(data) // 2] ^= 0x5A
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
