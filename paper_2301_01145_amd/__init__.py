"""hipoisson: spectral Poisson solves on MI355X through a C-ABI HIP library.

`Solver` wraps one plan for torch tensors on the GPU: device pointers and the
current HIP stream are handed to libhipoisson.so, which runs every step of the
solve.  The C functions are re-exported under their C names (module _lib).
"""
from . import _lib
from ._lib import (  # noqa: F401  (C-ABI names)
    HipoissonError, hp_bind_gradient, hp_bind_output, hp_desc, hp_get_gradient, hp_get_output,
    hp_input_shape, hp_last_error, hp_output_shape, hp_plan_create, hp_plan_create_batched,
    hp_plan_destroy, hp_query, hp_set_boundary, hp_set_input, hp_solve, hp_solve_adjoint,
    hp_autotune, hp_pass_stats, hp_set_timing, hp_status_string,
)

BCS = {"periodic": _lib.HP_PERIODIC, "dirichlet": _lib.HP_DIRICHLET,
       "neumann": _lib.HP_NEUMANN, "unbounded": _lib.HP_UNBOUNDED}
GRIDS = {"regular": _lib.HP_REGULAR, "staggered": _lib.HP_STAGGERED}
KERNELS = {"ps": _lib.HP_OP_PS, "fd2": _lib.HP_OP_FD2, "g2": _lib.HP_G_GAUSS2,
           "g4": _lib.HP_G_GAUSS4, "g6": _lib.HP_G_GAUSS6, "g8": _lib.HP_G_GAUSS8,
           "g10": _lib.HP_G_GAUSS10, "spectral": _lib.HP_G_SPECTRAL}
DIFFS = {"none": _lib.HP_D_NONE, "grad": _lib.HP_D_GRAD, "curl": _lib.HP_D_CURL,
         "div": _lib.HP_D_DIV, "nabla": _lib.HP_D_NABLA}


def make_desc(bc, grid, nc, lo=None, hi=None, kernel=None, diff="none", prec="f32", ncomp=1,
              inhomogeneous=False, sigma_cells=0.0):
    """Build an hp_desc from readable options (see include/hipoisson.h).  bc is
    one name for every face, or one name per axis ("periodic", "dirichlet",
    "neumann") for a mixed-boundary plan."""
    nd = len(nc)
    lo = list(lo) if lo is not None else [0.0] * nd
    hi = list(hi) if hi is not None else [1.0] * nd
    if kernel is None:
        kernel = "g2" if bc == "unbounded" else "ps"
    d = hp_desc()
    d.ndim = nd
    d.ncomp = ncomp
    for a in range(3):
        d.nc[a] = int(nc[a]) if a < nd else 1
        d.lo[a] = float(lo[a]) if a < nd else 0.0
        d.hi[a] = float(hi[a]) if a < nd else 1.0
    if isinstance(bc, (list, tuple)):
        if len(bc) != nd:
            raise ValueError("one boundary condition per axis")
        d.bc = _lib.HP_MIXED
        for a in range(nd):
            d.bc_axis[a] = BCS[bc[a]]
    else:
        d.bc = BCS[bc]
    d.grid = GRIDS[grid]
    d.kernel = KERNELS[kernel]
    d.diff = DIFFS[diff]
    d.prec = {"f32": _lib.HP_F32, "f64": _lib.HP_F64}[prec]
    d.inhomogeneous = int(bool(inhomogeneous))
    d.reg_sigma_cells = float(sigma_cells)
    return d


class Solver:
    """One plan for torch tensors (float32 or float64) on a ROCm device."""

    def __init__(self, bc, grid, nc, lo=None, hi=None, kernel=None, diff="none",
                 dtype=None, ncomp=1, inhomogeneous=False, sigma_cells=0.0, device="cuda"):
        import torch
        dtype = dtype or torch.float32
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be float32 or float64")
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.desc = make_desc(bc, grid, nc, lo, hi, kernel, diff,
                              "f32" if dtype == torch.float32 else "f64", ncomp,
                              inhomogeneous, sigma_cells)
        self.nd = len(nc)
        self.ncomp = ncomp
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.plan = hp_plan_create(self.desc, self.stream.cuda_stream)
        self.in_shape = tuple(hp_input_shape(self.plan)[:self.nd])
        self.out_shape = tuple(hp_output_shape(self.plan)[:self.nd])
        self.nderiv = int(hp_query(self.plan, _lib.HP_Q_NUM_DERIVS))
        self.inhomogeneous = bool(inhomogeneous)

    # -- helpers
    def _check_tensor(self, t, shape, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != self.dtype:
            raise ValueError(f"{name} must be a {self.dtype} tensor on {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def empty_output(self):
        import torch
        return torch.empty(self.out_shape, dtype=self.dtype, device=self.device)

    def model_bytes(self):
        return hp_query(self.plan, _lib.HP_Q_MODEL_BYTES)

    def passes(self):
        """Kernel launches of one solve."""
        return hp_query(self.plan, _lib.HP_Q_NUM_PASSES)

    def zero_mode(self):
        """Part of the bound source that the k = 0 projection removes (periodic and
        Neumann plans; 0 for a compatible source and for other BCs)."""
        return hp_query(self.plan, _lib.HP_Q_ZERO_MODE)

    def autotune(self, reps=5):
        """Time the kernel configurations of this plan and keep the fastest
        (hp_autotune); returns (tuned pass signatures, solve ms with the defaults,
        solve ms with the kept configuration), as measured while tuning."""
        hp_autotune(self.plan, reps)
        return (int(hp_query(self.plan, _lib.HP_Q_TUNED_PASSES)),
                hp_query(self.plan, _lib.HP_Q_TUNE_DEFAULT_MS),
                hp_query(self.plan, _lib.HP_Q_TUNE_BEST_MS))

    def bind(self, f, faces=None, psi=None, derivs=None):
        """Bind input, boundary and output tensors (no copies)."""
        comps = [f] if self.ncomp == 1 else list(f)
        for c, t in enumerate(comps):
            self._check_tensor(t, self.in_shape, "f")
            hp_set_input(self.plan, 0, c, t.data_ptr(), 1)
        if self.inhomogeneous:
            # {(axis, side): g} for every component, or one such dict per component
            faces = faces or {}
            per = list(faces) if isinstance(faces, (list, tuple)) else [faces] * self.ncomp
            if len(per) != self.ncomp:
                raise ValueError(f"faces: one dict per component ({self.ncomp}) or one for all")
            for c in range(self.ncomp):
                for a in range(self.nd):
                    shp = tuple(self.out_shape[b] for b in range(self.nd) if b != a)
                    for s in (0, 1):
                        g = (per[c] or {}).get((a, s))
                        if g is not None:
                            self._check_tensor(g, shp, f"face {(a, s)} of component {c}")
                        hp_set_boundary(self.plan, 0, a, s, c, g.data_ptr() if g is not None else None, 1)
        psi = psi if psi is not None else [self.empty_output() for _ in range(self.ncomp)]
        psi = [psi] if not isinstance(psi, (list, tuple)) else list(psi)
        for c, t in enumerate(psi):
            self._check_tensor(t, self.out_shape, "psi")
            hp_bind_output(self.plan, 0, c, t.data_ptr())
        derivs = derivs if derivs is not None else [self.empty_output() for _ in range(self.nderiv)]
        for c, t in enumerate(derivs):
            self._check_tensor(t, self.out_shape, "deriv")
            hp_bind_gradient(self.plan, 0, c, t.data_ptr())
        # the plan holds raw device pointers: keep every bound tensor alive for
        # as long as the binding stands (a freed block can be returned to the
        # driver, e.g. by torch.cuda.empty_cache, and a later solve would then
        # touch unmapped memory)
        self._keep = (comps, faces, psi, list(derivs))
        return psi, list(derivs)

    def run(self):
        """Launch the bound solve on the plan's stream."""
        hp_solve(self.plan)

    def solve(self, f, faces=None, psi=None, derivs=None):
        """Solve lap(psi) = f.  Returns (psi, derivs) as lists of tensors."""
        psi, derivs = self.bind(f, faces, psi, derivs)
        hp_solve(self.plan)
        self._keep = (f, faces, psi, derivs)
        return psi, derivs

    def adjoint(self, g_psi=None, g_derivs=None, grad_f=None):
        """Transpose of f -> (psi, derivs): returns grad_f (list per component)."""
        import torch
        grad_f = grad_f or [torch.empty(self.in_shape, dtype=self.dtype, device=self.device)
                            for _ in range(self.ncomp)]
        for c, t in enumerate(grad_f):
            self._check_tensor(t, self.in_shape, "grad_f")
            hp_set_input(self.plan, 0, c, t.data_ptr(), 1)
        gp = list(g_psi) if g_psi is not None else [None] * self.ncomp
        for c in range(self.ncomp):
            t = gp[c]
            if t is not None:
                self._check_tensor(t, self.out_shape, "g_psi")
            hp_bind_output(self.plan, 0, c, t.data_ptr() if t is not None else None)
        gd = list(g_derivs) if g_derivs is not None else [None] * self.nderiv
        for c in range(self.nderiv):
            t = gd[c]
            if t is not None:
                self._check_tensor(t, self.out_shape, "g_deriv")
            hp_bind_gradient(self.plan, 0, c, t.data_ptr() if t is not None else None)
        self._keep = (grad_f, gp, gd)  # bound before the launch reads them
        hp_solve_adjoint(self.plan)
        return grad_f

    def close(self):
        if getattr(self, "plan", None):
            hp_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
