"""Pins of the oracle's two-site measures (Eq. res:negativity,
Eq. metrics:fidelity) against closed forms: Bell and Werner states,
product states, pure-state overlaps, commuting (classical) fidelity, and the
symmetries the definitions imply."""
import numpy as np
import pytest

from oracle.dense import fidelity, negativity, partial_transpose_b


def _ket(*amps):
    v = np.array(amps, complex)
    return v / np.linalg.norm(v)


def _proj(v):
    return np.outer(v, v.conj())


SINGLET = _ket(0, 1, -1, 0)     # basis (p_i p_j) = 00, 01, 10, 11


def _random_rho(rng, rank=4):
    X = rng.standard_normal((4, rank)) + 1j * rng.standard_normal((4, rank))
    r = X @ X.conj().T
    return r / np.trace(r)


@pytest.mark.parametrize("p", [0.0, 0.2, 1 / 3, 0.5, 0.8, 1.0])
def test_negativity_of_werner_states(p):
    """rho = p |singlet><singlet| + (1 - p) I / 4: the partial transpose has
    eigenvalues (1 + p) / 4 (three times) and (1 - 3p) / 4, so the negativity
    is max(0, (3p - 1) / 4); 1/2 for the singlet itself."""
    rho = p * _proj(SINGLET) + (1 - p) * np.eye(4) / 4
    assert abs(negativity(rho) - max(0.0, (3 * p - 1) / 4)) < 1e-14


def test_negativity_of_product_and_scaled_states():
    rng = np.random.default_rng(3)
    a, b = _random_rho(rng)[:2, :2], _random_rho(rng)[:2, :2]
    a, b = a / np.trace(a), b / np.trace(b)
    assert abs(negativity(np.kron(a, b))) < 1e-14            # separable
    rho = _random_rho(rng)
    assert abs(negativity(7.5 * rho) - negativity(rho)) < 1e-14   # trace normalised
    # transposing site A instead of B gives the same spectrum
    pta = rho.reshape(2, 2, 2, 2).transpose(2, 1, 0, 3).reshape(4, 4)
    assert np.allclose(np.sort(np.linalg.eigvalsh(pta)),
                       np.sort(np.linalg.eigvalsh(partial_transpose_b(rho))), atol=1e-14)


def test_fidelity_closed_forms():
    rng = np.random.default_rng(5)
    rho, sigma = _random_rho(rng), _random_rho(rng)
    assert abs(fidelity(rho, rho) - 1.0) < 1e-12
    assert abs(fidelity(rho, sigma) - fidelity(sigma, rho)) < 1e-12
    U, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    assert abs(fidelity(U @ rho @ U.conj().T, U @ sigma @ U.conj().T) - fidelity(rho, sigma)) < 1e-12
    # pure states: |<psi|phi>|^2
    psi, phi = _ket(*(rng.standard_normal(4) + 1j * rng.standard_normal(4))), \
        _ket(*(rng.standard_normal(4) + 1j * rng.standard_normal(4)))
    assert abs(fidelity(_proj(psi), _proj(phi)) - abs(np.vdot(psi, phi)) ** 2) < 1e-7
    # commuting (diagonal) states: the classical fidelity (sum sqrt(p q))^2
    p, q = rng.random(4), rng.random(4)
    p, q = p / p.sum(), q / q.sum()
    assert abs(fidelity(np.diag(p), np.diag(q)) - np.sum(np.sqrt(p * q)) ** 2) < 1e-14
    assert 0.0 <= fidelity(rho, sigma) <= 1.0
