"""Seeded input generators: published generator values, determinism, shapes."""
import numpy as np

import fixtures as F


def test_splitmix64_published_vector():
    # splitmix64 seeded with 1234567, the reference sequence of its authors' generator
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [int(v) for v in F.splitmix64(1234567, 5)] == ref


def test_stream_is_batch_independent():
    a = F.Stream(9).uniform(10)
    s = F.Stream(9)
    b = np.concatenate([s.uniform(3), s.uniform(7)])
    np.testing.assert_array_equal(a, b)
    n = F.Stream(5).normal(200000)
    assert abs(n.mean()) < 0.01 and abs(n.std() - 1) < 0.01


def test_workload_shapes_and_media():
    w = F.c1()
    c = F.medium(w)
    assert c.shape == (128, 128) and c.dtype == np.float32
    assert 1500.0 <= c.min() and c.max() < 2200.0
    w2 = F.c2()
    c2 = F.medium(w2)
    assert c2.shape == (256, 512) and abs(c2.min() - 1500) < 1e-3 and abs(c2.max() - 4000) < 1e-3
    assert w2.prop_shape == (296, 552) and w2.ns == 64 and w2.nr == 256
    assert w2.cell_steps == 552 * 296 * 3000 * 64
    y = F.trials(w)[0]
    assert y.shape == (128, 128) and abs(np.abs(y).max() - 1.0) < 1e-7
    assert np.unravel_index(np.abs(y).argmax(), y.shape)[0] >= 5   # centres lie below the surface rows
    r = F.reflectivity(w2, c2)
    assert r.shape == (256, 512) and np.abs(r).max() > 0
