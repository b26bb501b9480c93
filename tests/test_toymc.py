"""Pins of the input generator: the drift of a hit is the true 3-D
closest distance between the helix and the wire (the paper's hit
definition, Sec. 3.2), checked by dense sampling of the helix arc; the
vectorised search agrees with the scalar one; event composition."""
import math

import numpy as np

from paper_2401_04576_amd import toymc


def test_drift_is_closest_distance_by_dense_sampling():
    rng = np.random.default_rng(61)
    ch = toymc.CHAMBER
    for _ in range(8):
        p = toymc.draw_helix(rng)
        for (layer, j, d, s, zw, rank) in toymc.helix_hits_fast(p)[::4]:
            px, py, tx, ty = (float(v) for v in ch.wire_geometry(layer, j))
            ss = np.linspace(s - 0.05, s + 0.05, 20001)
            dd = min(toymc.helix_line_distance(p, x, px, py, tx, ty)[0] for x in ss[::50])
            fine = np.array([toymc.helix_line_distance(p, x, px, py, tx, ty)[0] for x in
                             np.linspace(s - 1e-4, s + 1e-4, 2001)])
            assert d <= dd + 1e-12 and d <= fine.min() + 1e-12
            assert abs(zw) <= ch.half_length


def test_vectorised_search_matches_scalar():
    rng = np.random.default_rng(62)
    for _ in range(15):
        p = toymc.draw_helix(rng)
        a, b = toymc.helix_hits(p), toymc.helix_hits_fast(p)
        assert [(h[0], h[1]) for h in a] == [(h[0], h[1]) for h in b]
        assert max(abs(x[2] - y[2]) for x, y in zip(a, b)) < 1e-12


def test_event_composition():
    ev = toymc.config_event(2, 5)
    sig = ev.owner >= 0
    assert sig.sum() >= 18 and (~sig).sum() == int(np.floor(0.2 * sig.sum() + 0.5))
    assert np.allclose(ev.hits["band"], 3 * 150e-6)
    hc = toymc.CHAMBER.half_cell(ev.layer)
    assert (ev.hits["drift"] >= 0).all() and (ev.hits["drift"] <= hc + 1e-15).all()
    ev4 = toymc.config_event(4, 3)
    assert 20 <= ev4.n_hits <= 200 and 1 <= ev4.truth.shape[0] <= 5
    # wires are distinct within an event
    keys = set(zip(ev4.layer.tolist(), ev4.wire.tolist()))
    assert len(keys) == ev4.n_hits
    # the same seed gives the same event
    assert np.array_equal(toymc.config_event(4, 3).hits, ev4.hits)
