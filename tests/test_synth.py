"""Seeded input generators: reproducibility, distributions, sentinels (CPU only)."""
import numpy as np

import synth


def test_reproducible_and_seed_separated():
    a = synth.matrix(synth.seed_for(1, 0, 0), 37, 5, 40)
    b = synth.matrix(synth.seed_for(1, 0, 0), 37, 5, 40)
    c = synth.matrix(synth.seed_for(1, 0, 1), 37, 5, 40)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    v = ~np.isnan(a)
    assert not np.array_equal(a[v], c[v])


def test_padding_sentinels():
    x = synth.matrix(7, 5, 4, 9)
    v = x.reshape(4, 9)
    assert np.all(np.isfinite(v[:, :5])) and np.all(np.isnan(v[:, 5:]))
    c = synth.matrix(7, 5, 4, 9, pad=synth.pad_c_value())
    assert np.all(c.view(np.uint64).reshape(4, 9)[:, 5:] == synth.PAD_C_BITS)


def test_distributions():
    u = synth.draw(synth.rng(1), 100000, "uniform")
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.02
    i = synth.draw(synth.rng(2), 100000, "int")
    assert set(np.unique(i)) == set(range(-8, 9))
    s = synth.draw(synth.rng(3), 100000, "scaled", phi=8)
    e = np.frexp(s[s != 0])[1]
    assert e.min() >= -8 - 60 and e.max() <= 9
    assert np.all(np.abs(s) < 2.0 ** 8)


def test_problem_shapes_and_ld_rules():
    p = synth.problem(2, 0, "T", "N", 4099, 4099, 8, ld_rule=synth.ld_round8, dist="zeros")
    assert p["lda"] == 8 and p["ldb"] == 8 and p["ldc"] == 4104
    assert p["A"].size == 8 * 4099
    assert synth.ld_round8(4099) == 4104 and synth.ld_round8(1024) == 1024


def test_log_uniform_int_range():
    x = synth.log_uniform_int(synth.rng(5), 16, 512, 200000)
    assert x.min() == 16 and x.max() == 512
    # log-uniform: about as many draws in [16, 32) as in [256, 512]
    lo = np.mean((x >= 16) & (x < 32))
    hi = np.mean((x >= 256) & (x <= 512))
    assert abs(lo - hi) < 0.02
