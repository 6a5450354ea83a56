"""A context bound to PyTorch's current HIP stream, with slots whose device
memory PyTorch allocates and lends to the library."""
import torch

from . import _lib as L


class Context:
    """Owns an lbm context.  All work is ordered on ``stream``, a PyTorch
    stream (default: a new stream of default priority on ``device``; the
    legacy default stream cannot be captured into HIP graphs)."""

    def __init__(self, device=0, hbm_budget=0, max_slots=1, stream=None, lend_memory=True):
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.Stream(device=self.device)
        self.stream = stream
        self.lend_memory = lend_memory
        self._buffers = {}
        self.h = L.lbm_create(self.device, stream.cuda_stream, hbm_budget, max_slots)
        self._shape = {}

    def close(self):
        if self.h is not None:
            L.lbm_destroy(self.h)
            self.h = None
            self._buffers.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- slots -------------------------------------------------------------
    def add(self, case=None, **kw):
        """Admits a cavity (dict of problem parameters and/or lbm_case fields)."""
        c = case if isinstance(case, L.lbm_case) else L.make_case(case, **kw)
        buf, nbytes = None, 0
        if self.lend_memory:
            nbytes = L.lbm_footprint(c)
            if nbytes == 0:
                L.lbm_derive(c)  # raises with the reason
            t = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
            ptr = t.data_ptr()
            off = (-ptr) % 256
            buf = ptr + off
        slot = L.lbm_set_case(self.h, c, buf, nbytes)
        if self.lend_memory:
            self._buffers[slot] = t
        self._shape[slot] = (c.nx, c.ny)
        return slot

    def release(self, slot):
        L.lbm_release(self.h, slot)
        self._buffers.pop(slot, None)
        self._shape.pop(slot, None)

    # -- hot path ----------------------------------------------------------
    def step(self, slot, n):
        L.lbm_step(self.h, slot, n)

    def step_many(self, slots, nsteps):
        L.lbm_step_many(self.h, slots, nsteps)

    def set_group_bytes(self, nbytes):
        L.lbm_set_group_bytes(self.h, nbytes)

    def reduce(self, slot, allow_unstable=False):
        return L.lbm_reduce(self.h, slot, allow_unstable)

    def fields(self, slot, mask=63):
        nx, ny = self._shape[slot]
        return L.lbm_fields(self.h, slot, nx, ny, mask)

    def fields_noalloc(self, slot, mask=63):
        nx, ny = self._shape[slot]
        return L.lbm_fields_noalloc(self.h, slot, nx, ny, mask)

    def stream_probe(self, nbytes, pattern, launches=40):
        return L.lbm_stream_probe(self.h, nbytes, pattern, launches)

    def state_load(self, slot, f, g):
        L.lbm_state_load(self.h, slot, f, g)

    def state_save(self, slot):
        nx, ny = self._shape[slot]
        return L.lbm_state_save(self.h, slot, nx, ny)

    def checkpoint(self, slot):
        return L.lbm_checkpoint_save(self.h, slot)

    def restore(self, slot, blob):
        L.lbm_checkpoint_load(self.h, slot, blob)

    def set_report(self, slot, every, capacity):
        L.lbm_set_report(self.h, slot, every, capacity)

    def series(self, slot):
        return L.lbm_series(self.h, slot)

    def set_launch(self, precision, bx, by, cpl, flags=L.LBM_LAUNCH_DEFAULT):
        L.lbm_set_launch(self.h, precision, bx, by, cpl, flags)

    def get_launch(self, precision):
        return L.lbm_get_launch(self.h, precision)

    def set_fusion(self, precision, steps_per_launch, segment_rows=None):
        L.lbm_set_fusion(self.h, precision, steps_per_launch, segment_rows)

    def get_fusion(self, precision):
        return L.lbm_get_fusion(self.h, precision)

    def autotune(self, precision, nx, ny, cache_path=None):
        L.lbm_autotune(self.h, precision, nx, ny, cache_path)

    def set_graph_chunk(self, chunk):
        L.lbm_set_graph_chunk(self.h, chunk)

    def sync(self):
        L.lbm_sync(self.h)

    def info(self, slot):
        return L.lbm_slot_info(self.h, slot)

    def slot_fusion(self, slot):
        return L.lbm_slot_fusion(self.h, slot)
