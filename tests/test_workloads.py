"""CPU checks of the seeded input generator: the differentiable (torch) kernel builder
agrees with the tabulated one, and its parameter derivatives with finite differences."""
import numpy as np
import pytest

from paper_2410_03632_amd import workloads as W

torch = pytest.importorskip("torch")


def _points():
    cfg = W.tiny_config(n_chi=24, n_R=12)
    chi = np.linspace(cfg.chi_min, cfg.chi_max, cfg.n_chi)
    R = np.linspace(cfg.R_min, 1.0, cfg.n_R)
    return chi, chi[:, None] * R[None, :]


def test_torch_kernels_match_tabulated_kernels():
    chi, chi2 = _points()
    bins = [("g", 700.0, 150.0), ("g", 1500.0, 200.0), ("s", 1200.0, 400.0), ("s", 2400.0, 400.0)]
    K1, K2 = W.kernels(bins, chi, chi2)
    c = torch.tensor([b[1] for b in bins], dtype=torch.float64)
    s = torch.tensor([b[2] for b in bins], dtype=torch.float64)
    T1, T2 = W.kernels_torch([b[0] for b in bins], c, s, chi, chi2)
    for i in range(len(bins)):
        scale = max(np.abs(K1[i]).max(), np.abs(K2[i]).max())
        assert np.abs(T1[i].numpy() - K1[i]).max() <= 1e-6 * scale
        assert np.abs(T2[i].numpy() - K2[i]).max() <= 1e-6 * scale


def test_torch_kernel_parameter_gradients():
    chi, chi2 = _points()
    kinds = ["g", "s"]
    theta = np.array([900.0, 1800.0, 150.0, 400.0])
    rng = np.random.default_rng(0)
    G1 = rng.standard_normal((2, chi.size))
    G2 = rng.standard_normal((2,) + chi2.shape)

    def L(th):
        K1, K2 = W.kernels_torch(kinds, th[:2], th[2:], chi, chi2)
        return (K1 * torch.as_tensor(G1)).sum() + (K2 * torch.as_tensor(G2)).sum()

    th = torch.tensor(theta, requires_grad=True)
    L(th).backward()
    for i in range(4):
        h = 1e-5 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (float(L(torch.tensor(tp))) - float(L(torch.tensor(tm)))) / (2 * h)
        assert abs(float(th.grad[i]) - fd) <= 1e-6 * abs(fd) + 1e-12, (i, float(th.grad[i]), fd)
