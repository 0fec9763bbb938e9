"""Grid geometry of the oracle: point counts, spacing and coordinates per axis.

Source: Section 2.3.2 ("Grid Type"), eq. (gridpos).  A grid has N_c cells on
[X_l, X_u]; H = (X_u - X_l) / N_c.  REGULAR puts the solution on cell
boundaries, X_i = X_l + i H; STAGGERED puts it on cell centres,
X_i = X_l + (i + 1/2) H, i = 0 .. N_c - 1.

The paper says the number of REGULAR points "changes depending on the type of
solver" without listing it.  The reading used here is the one under which the
"N" of Table 1 (tab:Bounded) equals the length of the transform that the table
pairs with that BC and grid (so that every Table 1 FD2 eigenpair is exact):

  BC         REGULAR (unknowns n)          STAGGERED (unknowns n)
  Dirichlet  interior nodes 1..N_c-1       N_c cell centres
             (N_c + 1 output nodes, the two boundary nodes carry the BC value)
  Neumann    all nodes 0..N_c (N_c + 1)    N_c cell centres
  Periodic   nodes 0..N_c-1 (X_u == X_l)   N_c cell centres
  Unbounded  nodes 0..N_c (N_c + 1)        N_c cell centres
"""
import numpy as np

BCS = ("periodic", "dirichlet", "neumann", "unbounded")
GRIDS = ("regular", "staggered")


def spacing(lo, hi, nc):
    """Cell size H = (X_u - X_l) / N_c (eq. gridpos)."""
    return (float(hi) - float(lo)) / int(nc)


def unknowns(bc, grid, nc):
    """Transform length n on one axis (table in the module docstring)."""
    nc = int(nc)
    if bc == "dirichlet":
        return nc - 1 if grid == "regular" else nc
    if bc == "neumann":
        return nc + 1 if grid == "regular" else nc
    if bc == "periodic":
        return nc
    if bc == "unbounded":
        return nc + 1 if grid == "regular" else nc
    raise ValueError(bc)


def output_points(bc, grid, nc):
    """Number of solution points written per axis.

    Equal to the unknown count except for REGULAR Dirichlet, whose two
    boundary nodes are part of the output and hold the boundary value.
    """
    if bc == "dirichlet" and grid == "regular":
        return int(nc) + 1
    return unknowns(bc, grid, nc)


def positions(bc, grid, lo, hi, nc):
    """Coordinates of the output points (eq. gridpos)."""
    h = spacing(lo, hi, nc)
    m = output_points(bc, grid, nc)
    i = np.arange(m, dtype=np.float64)
    if grid == "regular":
        return float(lo) + h * i
    return float(lo) + h * (i + 0.5)
