"""Many independent bounded solves in one persistent launch (hp_plan_create_batched)."""
from . import _lib
from ._lib import (hp_autotune, hp_bind_output, hp_input_shape, hp_output_shape,
                   hp_plan_create_batched, hp_plan_destroy, hp_query, hp_set_input, hp_solve)


class BatchedSolver:
    """One batched plan over problems that share bc / grid / kernel / precision.

    problems: list of dicts with keys nc, lo, hi (other keys as in make_desc).
    The first solve uploads the bound pointers; capture a hipGraph (e.g. with
    torch.cuda.graph) only after one solve with the final bindings.
    """

    def __init__(self, bc, grid, problems, kernel="ps", dtype=None, device="cuda"):
        import torch
        from . import make_desc
        dtype = dtype or torch.float32
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        prec = "f32" if dtype == torch.float32 else "f64"
        self.descs = [make_desc(bc, grid, p["nc"], p.get("lo"), p.get("hi"), kernel, "none", prec)
                      for p in problems]
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.plan = hp_plan_create_batched(self.descs, self.stream.cuda_stream)
        self.in_shapes = [tuple(hp_input_shape(self.plan, i)) for i in range(len(problems))]
        self.out_shapes = [tuple(hp_output_shape(self.plan, i)) for i in range(len(problems))]

    def bind(self, fs, psis=None):
        import torch
        if psis is None:
            psis = [torch.empty(s, dtype=self.dtype, device=self.device) for s in self.out_shapes]
        for i, (f, psi) in enumerate(zip(fs, psis)):
            if tuple(f.shape) != self.in_shapes[i] or not f.is_contiguous() or f.dtype != self.dtype:
                raise ValueError(f"input {i}: expected contiguous {self.dtype} {self.in_shapes[i]}")
            if tuple(psi.shape) != self.out_shapes[i] or not psi.is_contiguous():
                raise ValueError(f"output {i}: expected contiguous {self.out_shapes[i]}")
            hp_set_input(self.plan, i, 0, f.data_ptr(), 1)
            hp_bind_output(self.plan, i, 0, psi.data_ptr())
        self._keep = (fs, psis)
        return psis

    def run(self):
        hp_solve(self.plan)

    def autotune(self, reps=5):
        """Tune radix orders, tiles and the work-item size (hp_autotune); returns
        (tuned pass signatures, tiles per work item).  Run one solve before
        capturing the plan into a graph."""
        hp_autotune(self.plan, reps)
        return (int(hp_query(self.plan, _lib.HP_Q_TUNED_PASSES)),
                int(hp_query(self.plan, _lib.HP_Q_BATCH_TILES)))

    def wavefront_kernel(self):
        """True when the batch runs the wavefront-FFT tile bodies."""
        return bool(hp_query(self.plan, _lib.HP_Q_BATCH_KERNEL))

    def kernel_mode(self):
        """0: general passes in one persistent launch; 1: wavefront tile bodies in
        one persistent launch; 2: wavefront tile bodies, one launch per pass level."""
        return int(hp_query(self.plan, _lib.HP_Q_BATCH_KERNEL))

    def error_flag(self):
        return int(hp_query(self.plan, _lib.HP_Q_BATCH_ERROR))

    def model_bytes(self):
        return hp_query(self.plan, _lib.HP_Q_MODEL_BYTES)

    def close(self):
        if getattr(self, "plan", None):
            hp_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
