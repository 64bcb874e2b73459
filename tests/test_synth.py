"""The seeded input generator: the device assembly of the orbitals equals the
host evaluation (same draws, same per-axis factors)."""
import numpy as np

from paper_2208_06097_amd import synth


def test_fill_orbitals_device_matches_host():
    torch = __import__("pytest").importorskip("torch")
    host = synth.mini(seed=7)
    dev = synth.fill_orbitals_device(synth.mini(seed=7, with_phi=False), device="cpu", chunk=5)
    assert dev.dtype == torch.float64 and tuple(dev.shape) == host.phi.shape
    assert np.max(np.abs(dev.numpy() - host.phi)) < 1e-14
    # normalization h^3 sum phi^2 = 1 per orbital
    h3 = host.h ** 3
    assert np.allclose(h3 * np.sum(dev.numpy() ** 2, axis=(1, 2, 3)), 1.0, atol=1e-13)
