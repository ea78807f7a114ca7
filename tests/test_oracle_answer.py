"""Pins of the answer-string oracle against facts fixed by mathematics:
basis states are returned exactly, a product state's answer is its most
likely string, ties take the given draw, and the probability carried along
is the distribution's value at the returned string."""
import itertools

import numpy as np
import pytest

from oracle import answer, statevector


def test_basis_state_is_returned():
    for x in itertools.product((0, 1), repeat=5):
        psi = np.zeros((2,) * 5, dtype=np.complex128)
        psi[x] = 1.0
        bits, probs = answer.answer_string(psi, 1e-12, [0] * 5)
        assert tuple(bits) == x
        for b, (p0, p1) in zip(x, probs):
            assert (p0, p1) == ((1.0, 0.0) if b == 0 else (0.0, 1.0))


def test_product_state_gives_its_most_likely_string():
    rng = np.random.default_rng(4)
    for _ in range(20):
        th = rng.uniform(0, np.pi, size=6)
        th[np.abs(th - np.pi / 2) < 1e-3] += 0.01  # keep clear of exact ties
        psi = statevector.product_state([[np.cos(t / 2), np.sin(t / 2) * np.exp(1j * t)] for t in th])
        bits, _ = answer.answer_string(psi, 1e-12, [0] * 6)
        best = np.unravel_index(np.argmax(np.abs(psi) ** 2), psi.shape)
        assert tuple(bits) == tuple(int(b) for b in best)


@pytest.mark.parametrize("draw", [0, 1])
def test_bell_state_tie_takes_the_draw(draw):
    psi = np.zeros((2, 2), dtype=np.complex128)
    psi[0, 0] = psi[1, 1] = 1 / np.sqrt(2)
    bits, probs = answer.answer_string(psi, 1e-12, [draw, 1 - draw])
    assert bits == [draw, draw]  # the second qubit follows the first; its own draw is unused
    np.testing.assert_allclose(probs[0], (0.5, 0.5), atol=1e-15)


def test_carried_probability_is_the_strings_probability():
    n = 6
    gl = [("U1", q, -1, 0.0, 100 + q) for q in range(n)]
    gl += [("U2", q, q + 1, 0.0, 200 + q) for q in range(n - 1)]
    psi = statevector.run(n, gl)
    bits, probs = answer.answer_string(psi, 1e-12, [0] * n)
    final = probs[-1][bits[-1]]
    np.testing.assert_allclose(final, abs(psi[tuple(bits)]) ** 2, rtol=1e-12)
    # each step's pair sums to the previous step's chosen probability
    prev = 1.0
    for (p0, p1), b in zip(probs, bits):
        np.testing.assert_allclose(p0 + p1, prev, rtol=1e-12)
        prev = p0 if b == 0 else p1
