"""Named synthetic workloads (shapes, seeds, operators) of the benchmarks.

Each workload is a block-Arnoldi or block-column-QR run on a synthetic
operator.  Shapes follow the paper's experiments (Sec. 6) scaled to one
MI355X: the paper names no operator, so Dirichlet Laplacians stand in for it,
and Stewart matrices (Sec. 6.1) stand in for the ill-conditioned inputs.
"""

from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    name: str
    grid: tuple            # Laplacian grid dims (2D or 3D)
    shift: float           # diagonal shift added to the stencil
    s: int                 # block width
    steps: int             # block steps after the start block
    leaf_rows: int         # TSQR leaf height
    seed: int = 0          # start-block seed
    notes: str = ""

    @property
    def n(self):
        n = 1
        for d in self.grid:
            n *= d
        return n

    @property
    def k_max(self):
        return (self.steps + 1) * self.s


WORKLOADS = {
    # small case: 2D 100x100 Laplacian + 0.01 I, s=4, 10 steps, 10 leaves of 1000 rows
    "lap2d-100x100-s4": Workload("lap2d-100x100-s4", (100, 100), 0.01, 4, 10, 1000, 0,
                                 "plain FP64, small: oracle runs in seconds"),
    # headline case: 2D 4096x4096 Laplacian (n = 2^24), s=8, 30 steps, 4096-row leaves
    "lap2d-4096x4096-s8": Workload("lap2d-4096x4096-s8", (4096, 4096), 0.0, 8, 30, 4096, 0,
                                   "plain FP64 on one GPU, basis in locally orthogonal form"),
    # large block: 3D 7-point 256^3 (n = 2^24), s=32, 16 steps
    "lap3d-256-s32": Workload("lap3d-256-s32", (256, 256, 256), 0.0, 32, 16, 4096, 5,
                              "large block"),
}


def grid_for(n_target):
    """Nearly square 2D grid (nx, ny) with nx*ny close to n_target."""
    import math
    nx = max(1, int(round(math.sqrt(n_target))))
    ny = max(1, int(round(n_target / nx)))
    return nx, ny
