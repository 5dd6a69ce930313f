"""Seeded input generator: determinism and the workload recipe."""
import numpy as np

import gen


def test_same_seed_same_instance():
    a, b = gen.config(1), gen.config(1)
    assert a.digest() == b.digest()
    c = gen.generate(1000, 64, 64, 8, gen.CONFIG_SEED[1] + 100, pin_max=8)
    assert c.digest() != a.digest()


def test_config1_recipe(c1_instance):
    I = c1_instance
    pins = np.diff(I.net_node_ptr)
    assert I.num_nets == 1000 and pins.min() >= 2 and pins.max() <= 8
    assert I.node_x.min() >= 0 and I.node_x.max() < 64 and I.node_y.max() < 64
    caps = I.caps
    # H layers have no edge past the last column, V layers none past the last row
    assert (caps[:, -1, 0::2] == 0).all() and (caps[-1, :, 1::2] == 0).all()
    inner = caps[:-1, :-1, :]
    assert inner.min() >= 4 and inner.max() <= 12
    for i in range(I.num_nets):
        b0, b1 = I.net_node_ptr[i], I.net_node_ptr[i + 1]
        cells = set(zip(I.node_x[b0:b1].tolist(), I.node_y[b0:b1].tolist()))
        assert len(cells) == b1 - b0, "pins of a net are distinct GCells"
        assert I.node_flags[b0] == 2 and (I.node_flags[b0 + 1:b1] == 1).all()


def test_layer_rc_law():
    I = gen.generate(1, 4, 4, 12, 5)
    assert I.r_mohm.tolist() == [20000, 20000, 14000, 14000, 9800, 9800, 6860, 6860, 4802, 4802, 3361, 3361]
    assert I.c_af.tolist() == [200, 200, 140, 140, 98, 98, 69, 69, 48, 48, 34, 34]
    assert I.layer_dir.tolist() == [0, 1] * 6


def test_heavy_tailed_pin_law():
    I = gen.config(2, num_nets=40000)
    p = np.diff(I.net_node_ptr)
    assert abs((p == 2).mean() - 0.55) < 0.01
    assert abs(((p == 3) | (p == 4)).mean() - 0.30) < 0.01
    assert p.max() <= 64 and abs(p.mean() - 3.5) < 0.05


def test_counter_generator_is_splitmix64():
    # published splitmix64 reference outputs for seed 1234567 (Steele et al. algorithm)
    x = 1234567
    ref = []
    for _ in range(3):
        x = (x + 0x9E3779B97F4A7C15) & (2**64 - 1)
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2**64 - 1)
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2**64 - 1)
        ref.append(z ^ (z >> 31))
    assert gen.counter_u64(1234567, 3).tolist() == ref
