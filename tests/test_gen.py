"""Host checks of the synthetic input generator and the lag rule."""
import numpy as np
import torch

import gen


def test_log_spaced_lags_c2():
    lags = gen.log_spaced_lags(500, 50)
    assert len(lags) == 50 and lags[0] == 1 and lags[-1] == 500
    assert all(b > a for a, b in zip(lags, lags[1:]))
    assert lags[:27] == list(range(1, 28))
    assert lags[27:] == [31, 35, 40, 45, 51, 58, 66, 75, 85, 96, 109, 124, 141,
                         160, 181, 206, 234, 265, 301, 342, 388, 440, 500]


def test_power_of_two_lags():
    assert gen.power_of_two_lags(64) == [1, 2, 4, 8, 16, 32, 64]
    assert gen.power_of_two_lags(100) == [1, 2, 4, 8, 16, 32, 64]


def test_stack_is_seeded_and_typed():
    c = gen.config("c1", N=3)
    a = gen.make_stack(c, 5)
    b = gen.make_stack(c, 5)
    d = gen.make_stack(c, 6)
    assert a.dtype == torch.float32 and a.shape == (3, 128, 128)
    assert torch.equal(a, b) and not torch.equal(a, d)
    c2 = gen.config("c2", N=2, n=256)
    u = gen.make_stack(c2, 2)
    assert u.dtype == torch.uint16
    v = u.to(torch.int32)
    assert int(v.min()) >= 0 and int(v.max()) <= 4095


def test_field_has_unit_variance_and_zero_mean():
    c = gen.config("c1", N=1, eps=1.0, noise="none", n=64)
    f = gen.make_stack(c, 9, flat_beam=True).double()[0] / c["peak"] - 1.0
    assert abs(float(f.mean())) < 1e-9
    assert 0.3 < float(f.var()) < 3.0


def test_cosine_stack_has_unit_mean():
    f = gen.cosine_stack(16, 4, [(1, 2, 0.1, 0.3), (-3, 5, 0.2, 1.0)])
    assert np.allclose(f.reshape(4, -1).mean(axis=1), 1.0, atol=1e-14)
