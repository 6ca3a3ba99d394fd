"""The seeded input generators: the streamed source draws the same numbers as
the whole-field one, and the link generator's width gives the target plaquette."""
import numpy as np

from paper_1811_08488_amd import synth
from tests import lattice_helpers as H


def test_streamed_source_equals_whole_field():
    L, Ls = (6, 4, 4, 6), 4
    phi = synth.source(L, Ls, 2, 77)
    par = H.parity_of_lex(L)
    ev = np.zeros((2, int(np.prod(L)) // 2, Ls, 4, 3), complex)
    od = np.zeros_like(ev)
    for r, cb0, e, o in synth.source_cb_chunks(L, Ls, 2, 77, sites_per_chunk=40):
        ev[r, cb0:cb0 + len(e)] = e
        od[r, cb0:cb0 + len(o)] = o
    assert np.array_equal(ev, phi[:, par == 0]) and np.array_equal(od, phi[:, par == 1])


def test_links_unitary_and_plaquette():
    eps = synth.tuned_eps()
    U = synth.gauge_field((8, 8, 8, 8), eps, 777)
    eye = np.eye(3)
    assert np.allclose(U[:50] @ np.conj(np.swapaxes(U[:50], -1, -2)), eye, atol=1e-13)
    assert np.allclose(np.linalg.det(U[:50]), 1.0, atol=1e-12)
    assert abs(synth.plaquette(U, (8, 8, 8, 8)) - 0.6) < 2e-3
