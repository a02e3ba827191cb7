"""Seeded synthetic inputs for displacement-based probing.

Shared by the tests and the benchmark; used by both the GPU library's callers
and the oracle's.  It holds no arithmetic of the method itself: it only
draws gauge links and workload parameters.

The paper's experiments use an LQCD gauge ensemble (a 32^3 x 64 clover
configuration) that is not available here.  These synthetic lattices stand
in for it: a free scalar Laplacian and gauge-covariant 3-colour Laplacians
whose links are random SU(3) matrices near the identity,

    U = exp(i * eps * H),   H = (G + G^H)/2 - tr(G + G^H)/6 * I,
    G_ab = N(0,1) + i N(0,1)   (numpy PCG64, array order [mu][site][a][b]),

computed as Q diag(exp(i eps w)) Q^H from the eigen-decomposition of H.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def random_links(dims, eps: float, seed: int, nc: int = 3) -> np.ndarray:
    """complex128 [4, N, nc, nc] special-unitary links U = exp(i eps H)."""
    N = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((4, N, nc, nc), dtype=np.complex128)
    chunk = 1 << 18
    for mu in range(4):
        for s0 in range(0, N, chunk):
            n = min(chunk, N - s0)
            G = rng.standard_normal((n, nc, nc)) + 1j * rng.standard_normal((n, nc, nc))
            H = 0.5 * (G + np.conj(np.swapaxes(G, 1, 2)))
            tr = np.trace(H, axis1=1, axis2=2).real / nc
            H -= tr[:, None, None] * np.eye(nc)[None]
            w, Q = np.linalg.eigh(H)
            ph = np.exp(1j * eps * w)
            out[mu, s0:s0 + n] = (Q * ph[:, None, :]) @ np.conj(np.swapaxes(Q, 1, 2))
    return out


@dataclass
class Workload:
    """One lattice problem: operator, displacement, colouring and noise."""
    name: str
    dims: tuple
    nc: int
    m2: float
    eps: float | None          # None: free field (U = 1)
    link_seed: int | None
    p: int
    ks: tuple                  # colouring distances (several = nested levels)
    order: str                 # "natural", "redblack" or "best"
    noise: str                 # "real_z2", "z2_complex" or "z4"
    noise_seed: int
    dilute: bool
    tol: float
    precision: str             # inner solver storage: "f64", "f32" or "bf16"
    extra: dict = field(default_factory=dict)

    @property
    def volume(self) -> int:
        return int(np.prod(self.dims))

    def links(self):
        if self.eps is None:
            return None
        return random_links(self.dims, self.eps, self.link_seed, self.nc)


# The five lattice workloads: a tiny free field checked in closed form, a
# small gauge lattice solved in plain FP64, a 16^4 nested-level batched
# mixed-precision workload, an uneven batch of small lattices and a 32^4
# lattice with the adjoint gradient.
FREE_4 = Workload("free-4^4", (4, 4, 4, 4), 1, 0.5, None, None, 1, (2,), "best", "real_z2", 0,
                  False, 1e-12, "f64")
GAUGE_8 = Workload("gauge-8^4x3", (8, 8, 8, 8), 3, 0.1, 0.3, 1, 2, (4,), "best", "z2_complex",
                   0, True, 1e-10, "f64")
GAUGE_16 = Workload("gauge-16^4x3-nested", (16, 16, 16, 16), 3, 0.05, 0.4, 1, 4, (1, 2, 4, 8),
                    "natural", "z2_complex", 0, True, 1e-8, "f32")
GAUGE_32 = Workload("gauge-32^4x3-grad", (32, 32, 32, 32), 3, 0.01, 0.5, 1, 8, (8,), "best",
                    "z2_complex", 0, True, 1e-10, "f64")


def uneven_batch(n: int = 64, seed: int = 4):
    """The uneven batch: n gauge 3-colour instances with extents drawn from
    {4,6,8,10,12}^4, m2 ~ U[0.05,0.5], eps ~ U[0.2,0.5], p from {1,2,3},
    distance-4 colouring, instance i with links from seed 100+i and noise
    seed i.  Parameters come from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        dims = tuple(int(v) for v in rng.choice([4, 6, 8, 10, 12], size=4))
        m2 = float(rng.uniform(0.05, 0.5))
        eps = float(rng.uniform(0.2, 0.5))
        p = int(rng.choice([1, 2, 3]))
        out.append(Workload(f"batch-{i}", dims, 3, m2, eps, 100 + i, p, (4,), "best",
                            "z2_complex", i, True, 1e-8, "bf16"))
    return out


def free_field_trace(dims, m2: float, p: int, nc: int = 1):
    """Tr(P_p A^{-1}) and its m2-derivative for the free field, from the
    Fourier diagonalisation of the Laplacian (an independent closed form):
    nc * sum_k cos(k0 p) / lam(k), lam(k) = m2 + sum_mu 4 sin^2(k_mu / 2)."""
    ks = np.meshgrid(*[2 * np.pi * np.arange(D) / D for D in dims], indexing="ij")
    lam = m2 + sum(4 * np.sin(k / 2) ** 2 for k in ks)
    c = np.cos(ks[0] * p)
    return nc * float(np.sum(c / lam)), -nc * float(np.sum(c / lam ** 2))
