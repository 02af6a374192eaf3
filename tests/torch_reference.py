"""Plain differentiable PyTorch (CPU, float64) forward of the scheme, used only
as an independent reference gradient for the adjoint (autograd through a
converged Newton solve of the cubic)."""
import torch


def laplacian(phi, bc):
    """sum_k (phi_{+k} + phi_{-k} - 2 phi) with the BC's out-of-range rule:
    Neumann mirrors the node (0: HN), Dirichlet reads zero (1: HD), periodic
    wraps (2: P)."""
    out = torch.zeros_like(phi)
    for ax in range(phi.dim()):
        if bc == 2:
            lo = torch.roll(phi, 1, ax)
            hi = torch.roll(phi, -1, ax)
        else:
            n = phi.shape[ax]
            first = phi.narrow(ax, 0, 1)
            last = phi.narrow(ax, n - 1, 1)
            if bc == 1:
                first = torch.zeros_like(first)
                last = torch.zeros_like(last)
            lo = torch.cat([first, phi.narrow(ax, 0, n - 1)], ax)
            hi = torch.cat([phi.narrow(ax, 1, n - 1), last], ax)
        out = out + (hi + lo - 2 * phi)
    return out


def cubic_root(xi, h, iters=40):
    th = xi
    for _ in range(iters):
        th = th - (th + h * (th ** 3 - th) - xi) / (1 + h * (3 * th ** 2 - 1))
    return th


def forward(phi0, eps2, dt, dx, bc, nsteps):
    h = dt / 2
    kappa = eps2 * dt / (dx * dx)
    phi = phi0
    for _ in range(nsteps):
        xi = phi + kappa * laplacian(phi, bc) - h * (phi ** 3 - phi)
        phi = cubic_root(xi, h)
    return phi
