"""Python view of one fw_sim object: torch supplies the device workspace and
the stream, the HIP library does the work (include/fw25.h)."""
import ctypes

import numpy as np

from . import native
from .native import check, lib


def _ptr(arr):
    return ctypes.c_void_p(arr.ctypes.data)


def beta_from_b_over_a(b_over_a):
    """Nonlinearity coefficient of a fluid with parameter B/A: 1 + B/(2A)."""
    return 1.0 + np.asarray(b_over_a, dtype=np.float64) / 2.0


class Simulation:
    """Grid of one or more domains advancing together.

    shapes: [(nx, ny, nz), ...] with unused trailing dims 1.
    """

    def __init__(self, ndim, shapes, dx, dt, n_mech, pml_cells=0, pml_params=None, device=None):
        import torch
        self.torch = torch
        self.ndim = int(ndim)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.n_domains = len(self.shapes)
        self.dx, self.dt, self.n_mech = float(dx), float(dt), int(n_mech)
        shp = np.ascontiguousarray(np.array(self.shapes, dtype=np.int64).reshape(-1, 3))
        self._h = ctypes.c_void_p()
        pp = None
        if pml_params is not None:
            self._pml_params = np.ascontiguousarray(np.asarray(pml_params, dtype=np.float64))
            pp = _ptr(self._pml_params)
        check(lib.fw_create_grid(ctypes.byref(self._h), self.ndim, self.n_domains, _ptr(shp), self.dx, self.dt,
                                 self.n_mech, int(pml_cells), pp))
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = lib.fw_workspace_bytes(self._h)
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        check(lib.fw_bind_workspace(self._h, ctypes.c_void_p(base + off), int(nbytes)))
        self.n_rec = 0
        self.n_t_max = 0

    # --------------------------------------------------------------- api --
    def _stream(self, stream=None):
        s = self.torch.cuda.current_stream(self.device) if stream is None else stream
        return ctypes.c_void_p(s.cuda_stream)

    def set_media(self, class_maps, class_base, c, rho, beta, c_noise_amp=0.0, noise_seed=0):
        cls = np.ascontiguousarray(np.concatenate([np.asarray(m, dtype=np.uint8).reshape(-1) for m in class_maps]))
        base = np.ascontiguousarray(np.asarray(class_base, dtype=np.int32))
        c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
        beta = np.ascontiguousarray(np.asarray(beta, dtype=np.float64))
        check(lib.fw_set_media(self._h, _ptr(cls), _ptr(base), int(c.size), _ptr(c), _ptr(rho), _ptr(beta),
                               float(c_noise_amp), ctypes.c_uint64(int(noise_seed))))

    def set_relaxation_table(self, kappa, d, alpha):
        kappa = np.ascontiguousarray(np.asarray(kappa, dtype=np.float64))
        d = np.ascontiguousarray(np.asarray(d, dtype=np.float64))
        alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
        check(lib.fw_set_relaxation_table(self._h, int(kappa.shape[0]), _ptr(kappa), _ptr(d), _ptr(alpha)))

    def set_sources(self, domain, cell, wave_idx, waves):
        domain = np.ascontiguousarray(np.asarray(domain, dtype=np.int32).reshape(-1))
        cell = np.ascontiguousarray(np.asarray(cell, dtype=np.int64).reshape(-1))
        wave_idx = np.ascontiguousarray(np.asarray(wave_idx, dtype=np.int32).reshape(-1))
        waves = np.ascontiguousarray(np.asarray(waves, dtype=np.float32))
        if waves.ndim == 1:
            waves = waves[None, :]
        check(lib.fw_set_sources(self._h, int(cell.size), _ptr(domain), _ptr(cell), _ptr(wave_idx),
                                 int(waves.shape[0]), _ptr(waves), int(waves.shape[1])))

    def set_receivers(self, domain, cell, n_t_max, out=None):
        """Receivers; with out (a contiguous float32 tensor on the simulation's
        device, at least n_t_max x n_rec elements) the traces are recorded
        into it (fw_set_receivers_into) instead of a library buffer."""
        domain = np.ascontiguousarray(np.asarray(domain, dtype=np.int32).reshape(-1))
        cell = np.ascontiguousarray(np.asarray(cell, dtype=np.int64).reshape(-1))
        if out is None:
            check(lib.fw_set_receivers(self._h, int(cell.size), _ptr(domain), _ptr(cell), int(n_t_max)))
        else:
            if out.dtype != self.torch.float32 or not out.is_contiguous() or out.device != self.device:
                raise ValueError("out must be a contiguous float32 tensor on %s" % self.device)
            check(lib.fw_set_receivers_into(self._h, int(cell.size), _ptr(domain), _ptr(cell), int(n_t_max),
                                            ctypes.c_void_p(out.data_ptr()), int(out.numel())))
        self._trace_buf = out          # borrowed by the library while set
        self.n_rec = int(cell.size)
        self.n_t_max = int(n_t_max)

    def prepare(self):
        """Build the tile lists and capture the step graph now (fw_prepare),
        so that following step() calls only launch."""
        check(lib.fw_prepare(self._h))

    def step(self, n_steps, stream=None):
        check(lib.fw_step(self._h, int(n_steps), self._stream(stream)))

    def read_receivers(self, stream=None):
        out = np.zeros((self.n_t_max, self.n_rec), dtype=np.float32)
        if out.size:
            check(lib.fw_read_receivers(self._h, _ptr(out), int(out.size), 0, self._stream(stream)))
        return out

    def read_receivers_device(self, stream=None):
        out = self.torch.zeros((self.n_t_max, self.n_rec), dtype=self.torch.float32, device=self.device)
        if out.numel():
            check(lib.fw_read_receivers(self._h, ctypes.c_void_p(out.data_ptr()), int(out.numel()), 1,
                                        self._stream(stream)))
        return out

    def read_field(self, field=0, domain=0, device=False, stream=None):
        """One field of one domain (0 pressure, 1..3 velocity x/y/z), shaped
        (nz, ny, nx); a torch device tensor if device else a numpy array."""
        nx, ny, nz = self.shapes[domain]
        if device:
            out = self.torch.empty((nz, ny, nx), dtype=self.torch.float32, device=self.device)
            check(lib.fw_read_field(self._h, int(field), int(domain), ctypes.c_void_p(out.data_ptr()), 1,
                                    self._stream(stream)))
            return out
        out = np.empty((nz, ny, nx), dtype=np.float32)
        check(lib.fw_read_field(self._h, int(field), int(domain), _ptr(out), 0, self._stream(stream)))
        return out

    def reset(self, stream=None):
        check(lib.fw_reset_state(self._h, self._stream(stream)))

    def get_step(self):
        v = ctypes.c_int64()
        check(lib.fw_get_step(self._h, ctypes.byref(v)))
        return v.value

    def first_nonfinite_step(self, stream=None):
        """First trace row (0-based step) with a non-finite receiver value
        since the last reset, or -1 (checked by every step on the device)."""
        v = ctypes.c_int64()
        check(lib.fw_first_nonfinite_step(self._h, ctypes.byref(v), self._stream(stream)))
        return v.value

    def state_bytes(self):
        return int(lib.fw_state_bytes(self._h))

    def _check_state_buffer(self, buf):
        if (buf.device != self.device or not buf.is_contiguous()
                or buf.numel() * buf.element_size() < self.state_bytes()):
            raise ValueError("state buffer must be a contiguous device tensor of at least %d bytes on %s"
                             % (self.state_bytes(), self.device))

    def save_state(self, buf=None, stream=None):
        if buf is None:
            buf = self.torch.empty(self.state_bytes(), dtype=self.torch.uint8, device=self.device)
        self._check_state_buffer(buf)
        check(lib.fw_save_state(self._h, ctypes.c_void_p(buf.data_ptr()), self._stream(stream)))
        return buf

    def load_state(self, buf, stream=None):
        self._check_state_buffer(buf)
        check(lib.fw_load_state(self._h, ctypes.c_void_p(buf.data_ptr()), self._stream(stream)))

    def time_kernels(self, n_steps, stream=None):
        """Advance n_steps with per-kernel HIP events; returns the average
        milliseconds of (velocity, pressure, sources+receivers)."""
        out = np.zeros(3, dtype=np.float64)
        check(lib.fw_time_kernels(self._h, int(n_steps), self._stream(stream), _ptr(out)))
        return out

    def stream_probe(self, mode, order, reps=5, stream=None):
        """Average ms of the memory-traffic probe (see fw_stream_probe)."""
        out = np.zeros(1, dtype=np.float64)
        check(lib.fw_stream_probe(self._h, int(mode), int(order), int(reps), self._stream(stream), _ptr(out)))
        return float(out[0])

    def energy_step(self, stream=None, check_finite=True):
        """One full step that also returns, per domain, (E^{n+1/2}, max|p|,
        number of non-finite pressures) with FP64 sums."""
        out = np.zeros((self.n_domains, 3), dtype=np.float64)
        rc = lib.fw_energy_step(self._h, _ptr(out), self._stream(stream))
        if rc != native.FW_ENONFINITE or check_finite:
            check(rc)
        return out

    def energy_step_noalloc(self, stream=None, check_finite=True):
        """energy_step through the allocation-free entry point (library
        scratch of fixed size; the tile lists must exist, i.e. one step taken)."""
        out = np.zeros((self.n_domains, 3), dtype=np.float64)
        rc = lib.fw_energy_step_noalloc(self._h, _ptr(out), self._stream(stream))
        if rc != native.FW_ENONFINITE or check_finite:
            check(rc)
        return out

    # ------------------------------------------------------------ adjoint --
    def adjoint_workspace(self, n_steps, ckpt_every):
        nb = int(lib.fw_adjoint_workspace_bytes(self._h, int(n_steps), int(ckpt_every)))
        if nb < 0:
            raise native.FWError(native.FW_EINVAL, "bad adjoint workspace request")
        return self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)

    def forward_checkpointed(self, n_steps, ckpt_every, work, stream=None):
        """Reset, run n_steps and store checkpoints in work (see fw25.h)."""
        check(lib.fw_forward_checkpointed(self._h, int(n_steps), int(ckpt_every), ctypes.c_void_p(work.data_ptr()),
                                          int(work.numel()), self._stream(stream)))

    def _grad_buffer(self, g, ncell):
        torch = self.torch
        if g is None:
            return torch.zeros(ncell, dtype=torch.float32, device=self.device)
        if g.dtype != torch.float32 or not g.is_contiguous() or g.numel() != ncell or g.device != self.device:
            raise ValueError("gradient buffers must be contiguous float32 tensors of %d cells on %s"
                             % (ncell, self.device))
        return g

    def _adj_source(self, adj_src, n_steps):
        adj_src = adj_src.to(device=self.device, dtype=self.torch.float32).contiguous()
        if adj_src.numel() < min(int(n_steps), self.n_t_max) * self.n_rec:
            raise ValueError("adj_src needs [n_steps][n_rec] values")
        return adj_src

    def set_time_space_stencil(self, c_ref):
        """Staggered coefficients tuned to the speed c_ref (time-space-domain
        set of fw_set_time_space_stencil); 0 restores the Taylor set."""
        check(lib.fw_set_time_space_stencil(self._h, float(c_ref)))

    def set_widened_stencil(self, c_ref):
        """2D only: the widened stencil (fourth order in time in every
        direction) tuned to the speed c_ref; 0 restores the Taylor set."""
        check(lib.fw_set_widened_stencil(self._h, float(c_ref)))

    def stencil(self):
        """The staggered coefficients in use (FP64): ([c_1..c_4], b)."""
        out = (ctypes.c_double * 5)()
        check(lib.fw_get_stencil(self._h, out))
        return list(out)[:4], out[4]

    def set_strength_map(self, scale, stream=None):
        """Per-voxel relaxation strength scale s(x) in [0, 1] (a device float
        tensor over all cells, unpadded layout), or None to clear it.  The
        tensor is borrowed: the Simulation keeps a reference."""
        if scale is None:
            self._strength = None
            check(lib.fw_set_strength_map(self._h, None, self._stream(stream)))
            return
        ncell = sum(int(np.prod(s)) for s in self.shapes)
        t = scale.to(device=self.device, dtype=self.torch.float32).contiguous()
        if t.numel() != ncell:
            raise ValueError("the strength map needs %d values" % ncell)
        check(lib.fw_set_strength_map(self._h, ctypes.c_void_p(t.data_ptr()), self._stream(stream)))
        self._strength = t

    def set_class_alpha0(self, alpha0):
        """Power-law alpha0 per class (for dJ/dalpha0 of adjoint)."""
        a0 = np.ascontiguousarray(np.asarray(alpha0, dtype=np.float64).reshape(-1))
        check(lib.fw_set_class_alpha0(self._h, int(a0.size), _ptr(a0)))

    def adjoint(self, n_steps, ckpt_every, work, adj_src, grad_c=None, grad_alpha0=None, with_alpha0=True,
                stream=None):
        """Reverse sweep; adj_src is a device float tensor [n_steps][n_rec]
        (dJ/d trace).  Returns (dJ/dc, dJ/dalpha0) per cell, unpadded layout
        (dJ/dalpha0 is None when with_alpha0 is False)."""
        ncell = sum(int(np.prod(s)) for s in self.shapes)
        grad_c = self._grad_buffer(grad_c, ncell)
        if with_alpha0:
            grad_alpha0 = self._grad_buffer(grad_alpha0, ncell)
        adj_src = self._adj_source(adj_src, n_steps)
        check(lib.fw_adjoint(self._h, int(n_steps), int(ckpt_every), ctypes.c_void_p(work.data_ptr()),
                             int(work.numel()), ctypes.c_void_p(adj_src.data_ptr()),
                             ctypes.c_void_p(grad_c.data_ptr()),
                             ctypes.c_void_p(grad_alpha0.data_ptr() if with_alpha0 else None),
                             self._stream(stream)))
        return grad_c, (grad_alpha0 if with_alpha0 else None)

    def adjoint_modulus(self, n_steps, ckpt_every, work, adj_src, grad_K=None, grad_s=None, stream=None):
        """The same sweep before the chain rule: (dJ/dK, dJ/ds) per cell."""
        ncell = sum(int(np.prod(s)) for s in self.shapes)
        grad_K = self._grad_buffer(grad_K, ncell)
        grad_s = self._grad_buffer(grad_s, ncell)
        adj_src = self._adj_source(adj_src, n_steps)
        check(lib.fw_adjoint_modulus(self._h, int(n_steps), int(ckpt_every), ctypes.c_void_p(work.data_ptr()),
                                     int(work.numel()), ctypes.c_void_p(adj_src.data_ptr()),
                                     ctypes.c_void_p(grad_K.data_ptr()), ctypes.c_void_p(grad_s.data_ptr()),
                                     self._stream(stream)))
        return grad_K, grad_s

    def set_option(self, key, value):
        check(lib.fw_set_option(self._h, int(key), int(value)))

    def close(self):
        if self._h:
            lib.fw_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
