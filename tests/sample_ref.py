"""Reference values for the sampler tests, computed with numpy only (no
oracle, no GPU code): the Philox slots from numpy's own Philox4x64-10, the
closed-form draws of the tail-mass model, seeds that hit its bin boundaries,
and a pooled chi-square test."""
import numpy as np
from scipy import stats as sstats

U64 = np.uint64
ALL_ONES = np.full(4, 2**64 - 1, dtype=np.uint64)


def numpy_slots(seed, H, W):
    """(H, W, 3) slots from numpy's Philox: the stream starting before counter 0
    yields the blocks of counters 0, 1, 2, ... in turn."""
    g = np.random.Philox(key=np.array([seed, 0], dtype=U64), counter=ALL_ONES.copy())
    raw = g.random_raw(4 * H * W).reshape(H, W, 4)
    return (raw[:, :, :3] >> U64(48)).astype(np.int64)


def decrement(ctr):
    c = [int(v) for v in ctr]
    for i in range(4):
        c[i] = (c[i] - 1) % 2**64
        if c[i] != 2**64 - 1:
            break
    return np.array(c, dtype=U64)


def closed_form_delta(slots):
    """The delta model's draws: channel means -100, +100, -100 put F = 1
    (resp. 0) at every interior edge, so cdf_k = k + 65280 for k >= 1 in R
    and B (freq_0 = 65281, the rest 1) and cdf_k = k for k <= 255 in G
    (freq_255 = 65281)."""
    out = np.zeros(slots.shape, dtype=np.uint8)
    for c in (0, 2):
        s = slots[..., c]
        out[..., c] = np.where(s < 65281, 0, s - 65280)
    s = slots[..., 1]
    out[..., 1] = np.where(s < 255, s, 255)
    return out


def boundary_seeds(H=8, W=8):
    """Seeds whose H x W slots hit each bin boundary of the delta model
    exactly: R or B slot 65280 (last slot of bin 0) and 65281 (bin 1), G slot
    254 (bin 254) and 255 (first slot of bin 255). A pure function of the
    generator, so the search always returns the same seeds."""
    want = {(0, 65280): None, (0, 65281): None, (1, 254): None, (1, 255): None}
    for seed in range(1, 200000):
        s = numpy_slots(seed, H, W)
        rb = np.concatenate([s[..., 0].ravel(), s[..., 2].ravel()])
        for (ch, v) in want:
            if want[(ch, v)] is None and np.any((rb if ch == 0 else s[..., 1].ravel()) == v):
                want[(ch, v)] = seed
        if all(x is not None for x in want.values()):
            return want
    raise AssertionError("no boundary seeds found")


def chi2_pvalue(counts, pmf, min_expected=5.0):
    """Pearson chi-square, bins with expected count below min_expected pooled."""
    n = counts.sum()
    exp = pmf * n
    order = np.argsort(exp)
    obs_b, exp_b, acc_o, acc_e = [], [], 0.0, 0.0
    for k in order:
        acc_o += counts[k]
        acc_e += exp[k]
        if acc_e >= min_expected:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        obs_b[-1] += acc_o
        exp_b[-1] += acc_e
    obs_b, exp_b = np.array(obs_b), np.array(exp_b)
    chi2 = float(((obs_b - exp_b) ** 2 / exp_b).sum())
    return float(sstats.chi2.sf(chi2, len(obs_b) - 1)), len(obs_b)
