"""Named workloads: cluster model, size and tree-force parameters.

Softening follows the paper's standard value eps = 4/N (Table 1) and the
changeover ratio gamma = r_in / r_out = 0.1 (Section 2.1).  The neighbour
search radius is h = 1.1 * r_out for every workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .ic import Cluster, king, plummer, salpeter_masses


@dataclass(frozen=True)
class Workload:
    name: str
    model: str          # "plummer" | "king9"
    n: int
    imf: str            # "equal" | "salpeter"
    theta: float
    n_crit: int
    r_out: float
    gamma: float = 0.1
    h_factor: float = 1.1
    n_leaf: int = 16
    extra: dict = field(default_factory=dict)

    @property
    def eps(self) -> float:
        return 4.0 / self.n

    @property
    def r_in(self) -> float:
        return self.gamma * self.r_out

    @property
    def r_search(self) -> float:
        return self.h_factor * self.r_out

    def params(self, **over) -> dict:
        d = dict(eps=self.eps, r_in=self.r_in, r_out=self.r_out, theta=self.theta,
                 r_search=self.r_search, n_crit=self.n_crit, n_leaf=self.n_leaf,
                 use_quadrupole=1)
        d.update(over)
        return d


WORKLOADS = {
    # Plummer N=4096, equal mass, FP64 force + potential + neighbour lists.
    "plummer4k": Workload("plummer4k", "plummer", 4096, "equal", 0.5, 64, 0.01),
    # Plummer N=65536 with a Salpeter IMF [0.1, 100]: FP64 vs mixed precision.
    "plummer64k_salpeter": Workload("plummer64k_salpeter", "plummer", 65536, "salpeter",
                                    0.4, 128, 0.005),
    # King W0=9, N=2^20, equal mass: 16 leapfrog steps of dt = 1/256.
    "king9_1m": Workload("king9_1m", "king9", 1 << 20, "equal", 0.5, 256, 0.002,
                         extra={"steps": 16, "dt": 1.0 / 256}),
    # Plummer N=2^22 Salpeter: theta x n_crit sweep.
    "plummer4m_salpeter": Workload("plummer4m_salpeter", "plummer", 1 << 22, "salpeter",
                                   0.5, 128, 0.001,
                                   extra={"thetas": (0.3, 0.5, 0.7),
                                          "n_crits": (64, 128, 256, 512)}),
    # Plummer N=2^18 equal mass: FP32 forward + VJP.
    "plummer256k": Workload("plummer256k", "plummer", 1 << 18, "equal", 0.5, 128, 0.004),
}


def make_cluster(w: Workload | str, seed: int = 1, n: int | None = None) -> Cluster:
    """Draw the cluster of workload ``w`` (optionally at a different size ``n``)."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    n = w.n if n is None else n
    masses = salpeter_masses(n, seed + 1000) if w.imf == "salpeter" else None
    if w.model == "plummer":
        return plummer(n, seed, masses=masses)
    if w.model == "king9":
        c = king(n, 9.0, seed)
        return c
    raise ValueError(w.model)
