"""Seeded synthetic inputs shared by the tests, the oracle's callers and the bench.

This module only draws random numbers and lays them out; it holds none of the
operator's arithmetic (no derivative matrix, no geometry, no summation).

Layout of an "L-vector" (element-local storage, the data layout of every
vector that crosses the library boundary): shape ``(E, N+1, N+1, N+1)`` indexed
``[e, k, j, i]`` with ``i`` fastest in memory, and element index
``e = ex + nx*(ey + ny*ez)``.  Element ``(ex, ey, ez)``'s local node
``(i, j, k)`` sits on the global lattice point ``(ex*N+i, ey*N+j, ez*N+k)`` of
the ``(nx*N+1) x (ny*N+1) x (nz*N+1)`` box lattice.

The Nekbone problem is a 3-D Poisson equation on a box of E hexahedra with
(N+1)^3 nodes each (Sec. VIII-A); the random right-hand sides below are the
synthetic stand-in for its forcing.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "lattice_shape",
    "lattice_to_lvector",
    "random_lattice",
    "continuous_rhs",
    "iid_lvector",
    "log_uniform_box",
    "batch_instances",
    "poisson_arrivals",
    "serving_requests",
]


def lattice_shape(nx: int, ny: int, nz: int, N: int) -> tuple[int, int, int]:
    """Shape ``(NZ, NY, NX)`` of the global node lattice of a box mesh."""
    return (nz * N + 1, ny * N + 1, nx * N + 1)


def lattice_to_lvector(grid: np.ndarray, nx: int, ny: int, nz: int, N: int) -> np.ndarray:
    """Copy lattice values into element-local layout (pure strided gather).

    ``grid`` has shape ``(NZ, NY, NX)``; the result has shape
    ``(E, N+1, N+1, N+1)`` with ``out[e, k, j, i] = grid[ez*N+k, ey*N+j, ex*N+i]``.
    """
    n = N + 1
    win = np.lib.stride_tricks.sliding_window_view(grid, (n, n, n))[::N, ::N, ::N]
    assert win.shape == (nz, ny, nx, n, n, n)
    return np.array(win, copy=True).reshape(nx * ny * nz, n, n, n)  # own, writable memory


def random_lattice(seed: int, nx: int, ny: int, nz: int, N: int, zero_boundary: bool = True) -> np.ndarray:
    """iid uniform[-1, 1] per lattice node from ``default_rng(seed)`` (PCG64).

    With ``zero_boundary`` the nodes on the box faces are set to 0, the
    structure of a field with homogeneous Dirichlet data.
    """
    rng = np.random.default_rng(seed)
    g = rng.uniform(-1.0, 1.0, size=lattice_shape(nx, ny, nz, N))
    if zero_boundary:
        g[0, :, :] = 0.0
        g[-1, :, :] = 0.0
        g[:, 0, :] = 0.0
        g[:, -1, :] = 0.0
        g[:, :, 0] = 0.0
        g[:, :, -1] = 0.0
    return g


def continuous_rhs(seed: int, nx: int, ny: int, nz: int, N: int, zero_boundary: bool = True) -> np.ndarray:
    """Continuous L-vector: one uniform[-1,1] draw per global node, copied to
    every element that holds that node.  Flat float64 array of length L."""
    g = random_lattice(seed, nx, ny, nz, N, zero_boundary)
    return np.ascontiguousarray(lattice_to_lvector(g, nx, ny, nz, N).reshape(-1))


def iid_lvector(seed: int, L: int) -> np.ndarray:
    """Discontinuous L-vector: iid uniform[-1,1] per element-local entry."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=L)


def log_uniform_box(rng: np.random.Generator, lo: int, hi: int) -> tuple[int, int, int]:
    """Box shape with element count near a log-uniform draw in [lo, hi].

    T = exp(U[ln lo, ln hi]); nx = round(T^(1/3)); ny = round(sqrt(T/nx));
    nz = max(1, round(T/(nx*ny))); the realised E = nx*ny*nz is then clamped
    into [lo, hi] by shrinking or growing nz.
    """
    T = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    nx = max(1, int(round(T ** (1.0 / 3.0))))
    ny = max(1, int(round(math.sqrt(T / nx))))
    nz = max(1, int(round(T / (nx * ny))))
    while nx * ny * nz > hi and nz > 1:
        nz -= 1
    while nx * ny * nz < lo:
        nz += 1
    return nx, ny, nz


def batch_instances(seed: int = 1000, count: int = 256, e_lo: int = 64, e_hi: int = 4096,
                    orders=(3, 5, 7, 9, 11)) -> list[dict]:
    """Independent solve instances of the batching workload.

    Instance i draws from ``default_rng(seed + i)``: a log-uniform box in
    [e_lo, e_hi] elements, an order uniform over ``orders``, a deformation
    amplitude 0.05*U(0.5, 1) and a right-hand-side seed.
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        nx, ny, nz = log_uniform_box(rng, e_lo, e_hi)
        N = int(orders[int(rng.integers(0, len(orders)))])
        amp = 0.05 * float(rng.uniform(0.5, 1.0))
        out.append(dict(index=i, nx=nx, ny=ny, nz=nz, N=N, amp=amp,
                        rhs_seed=int(seed + i) * 7919 + 11))
    return out


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def serving_requests(seed: int, count: int, e_lo: int = 64, e_hi: int = 32768,
                     orders=(5, 7, 9), amp: float = 0.05) -> list[dict]:
    """Solve requests of the serving workload: log-uniform boxes, uniform order."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx, ny, nz = log_uniform_box(rng, e_lo, e_hi)
        N = int(orders[int(rng.integers(0, len(orders)))])
        out.append(dict(index=i, nx=nx, ny=ny, nz=nz, N=N, amp=amp,
                        rhs_seed=int(seed) * 100003 + i))
    return out


def continuous_rhs_device(seed: int, nx: int, ny: int, nz: int, N: int, device, zero_boundary: bool = True):
    """A continuous right-hand side drawn on the GPU (for serving, where a
    request's data must not wait on the host): uniform[-1,1] per lattice node
    from torch's Philox generator seeded with ``seed``, zero on the box faces,
    copied into element-local layout by a strided window view.  Returns a
    float64 CUDA tensor of length L."""
    import torch

    n = N + 1
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    g = torch.rand(lattice_shape(nx, ny, nz, N), generator=gen, device=device, dtype=torch.float64)
    g = g * 2.0 - 1.0
    if zero_boundary:
        g[0], g[-1] = 0.0, 0.0
        g[:, 0], g[:, -1] = 0.0, 0.0
        g[:, :, 0], g[:, :, -1] = 0.0, 0.0
    win = g.unfold(0, n, N).unfold(1, n, N).unfold(2, n, N)  # (nz, ny, nx, k, j, i)
    return win.contiguous().reshape(-1)
