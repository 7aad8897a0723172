"""Seeded input generators (CPU): determinism, column-subset regeneration,
planted structure and density recipes."""
import math

import numpy as np
import torch

from paper_2411_19702_amd import synth


def test_hash_matches_reference_lowbias32():
    # lowbias32 written out with Python ints (unbounded) vs the split-multiply tensor form.
    def lb(x):
        x ^= x >> 16
        x = (x * 0x7FEB352D) & 0xFFFFFFFF
        x ^= x >> 15
        x = (x * 0x846CA68B) & 0xFFFFFFFF
        x ^= x >> 16
        return x
    xs = [0, 1, 2, 0xDEADBEEF, 0xFFFFFFFF, 123456789]
    got = synth._lowbias32(torch.tensor(xs, dtype=torch.int64)).tolist()
    assert got == [lb(x) for x in xs]


def test_generate_is_deterministic_and_binary():
    spec = synth.spec_small()
    a = synth.generate(spec)
    b = synth.generate(spec, row_chunk=77)
    assert a.dtype == torch.uint8 and a.shape == (1000, 200)
    assert torch.equal(a, b)
    assert set(torch.unique(a).tolist()) <= {0, 1}


def test_columns_subset_equals_full_matrix_columns():
    spec = synth.spec_mid(m=3000)
    full = synth.generate(spec)
    cols = [0, 5, spec.planted[0][0], spec.derived[0][0], spec.derived[-1][0], 1023]
    sub = synth.columns(spec, cols, row_chunk=1000)
    assert torch.equal(sub, full[:, cols])


def test_planted_and_derived_structure():
    spec = synth.spec_mid(m=20000)
    X = synth.generate(spec).numpy()
    for dst, src, q in spec.planted[:8]:
        flips = np.mean(X[:, dst] != X[:, src])
        assert abs(flips - q) < 0.02, (dst, src, q, flips)
    for dst, a, b, op in spec.derived:
        want = (X[:, a] & X[:, b]) if op == "and" else (X[:, a] ^ X[:, b])
        assert np.array_equal(X[:, dst], want)


def test_density_recipes():
    s3 = synth.spec_large()
    assert s3.p.min() >= 0.001 - 1e-12 and s3.p.max() <= 0.2 + 1e-12
    X = synth.columns(s3, list(range(0, 4096, 512)), row_chunk=1 << 18)
    dens = X.float().mean(dim=0).numpy()
    assert np.allclose(dens, s3.p[::512], atol=0.003)
    s2 = synth.spec_mid()
    assert s2.p.min() >= 0.005 and s2.p.max() <= 0.95
    assert len(s2.planted) == 64 and len(s2.derived) == 32


def test_padded_pitch_zero_fill():
    spec = synth.spec_random(9, 50, 13, ldx=32)
    X = synth.generate(spec)
    assert X.shape == (50, 32)
    assert int(X[:, 13:].sum()) == 0


def test_batched_and_served_recipes():
    specs = synth.specs_batched(count=16)
    for s in specs:
        assert 500 <= s.m <= 50_000 and 64 <= s.n <= 2048
        assert len(s.planted) == min(int(math.floor(0.05 * s.n)), s.n // 2)
    reqs = synth.request_trace(count=20, qps=10.0)
    t = [r.arrival_s for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    for r in reqs:
        assert 1000 <= r.spec.m <= 200_000 and 128 <= r.spec.n <= 8192


def test_categorical_generators():
    spec = synth.spec_categorical(3, 700, 25, 1, 9, planted=3)
    X = synth.cat_generate(spec).numpy()
    assert X.shape == (700, 25)
    assert (X < spec.levels[None, :]).all()
    cols = [0, 7, 24, 3]
    assert np.array_equal(synth.cat_columns(spec, cols).numpy(), X[:, cols])
    assert np.array_equal(synth.cat_generate(spec).numpy(), X)          # deterministic
    for dst, src, q in spec.planted:                                     # copies agree on most rows
        agree = np.mean(X[:, dst] == X[:, src] % spec.levels[dst])
        assert agree > 1 - q - 0.1, (dst, src, q, agree)
    g = synth.spec_genotypes(m=20000, v=40)
    G = synth.cat_generate(g).numpy()
    assert set(np.unique(G)) <= {0, 1, 2} and (g.levels == 3).all()
    f = g.cum[:, 0]                                                      # P(code 0) = (1 - maf)^2
    assert np.allclose(np.mean(G == 0, axis=0), f, atol=0.02)
    padded = synth.cat_generate(synth.spec_categorical(4, 50, 10, ldx=16)).numpy()
    assert padded.shape == (50, 16) and (padded[:, 10:] == 0).all()
