"""Python front end of the C ABI: argument marshalling only.

PyTorch supplies device memory (byte tensors) and the stream; every step of
the method runs in the HIP kernels of liblbmhd.so.
"""

from __future__ import annotations

import ctypes

from . import native as N

_DTYPES = {"fp64": N.LBM_FP64, "fp32": N.LBM_FP32, "fp16": N.LBM_FP16, "bf16": N.LBM_BF16}
_STENCILS = {"iso9": N.LBM_STENCIL_ISO9, "central5": N.LBM_STENCIL_CENTRAL5,
             "local_iso9": N.LBM_STENCIL_LOCAL_ISO9, "local_central5": N.LBM_STENCIL_LOCAL_CENTRAL5}
_SCHEDULES = {"fused": N.LBM_SCHED_FUSED, "aa": N.LBM_SCHED_AA, "aa_lagged": N.LBM_SCHED_AA_LAGGED}
_CLOSURES = {"analytic": N.LBM_CLOSURE_ANALYTIC, "learned": N.LBM_CLOSURE_LEARNED, "full": N.LBM_CLOSURE_FULL}
_MAG = {"d2q5": N.LBM_MAG_D2Q5, "d2q9": N.LBM_MAG_D2Q9}


def make_params(nx, ny, nu, eta, delta=0.0, closure_scale=1.0, s5=0.0, s6=0.0, s7=0.0, s8=0.0,
                grad_stencil="iso9", dtype="fp64", schedule="fused", rho0=1.0, b_ref=(0.0, 0.0),
                closure="analytic", mag_lattice="d2q5") -> N.LbmParams:
    return N.LbmParams(
        nx=int(nx), ny=int(ny), nu=float(nu), eta=float(eta),
        s5=float(s5 or 0.0), s6=float(s6 or 0.0), s7=float(s7 or 0.0), s8=float(s8 or 0.0),
        delta=float(delta), closure_scale=float(closure_scale),
        grad_stencil=_STENCILS[grad_stencil], dtype=_DTYPES[dtype],
        schedule=_SCHEDULES[schedule], closure=_CLOSURES[closure], mag_lattice=_MAG[mag_lattice], reserved=0,
        rho0=float(rho0),
        bref_x=float(b_ref[0]), bref_y=float(b_ref[1]))


def state_bytes(params: N.LbmParams) -> int:
    return N.load().lbm_state_bytes(ctypes.byref(params))


def work_bytes(params: N.LbmParams) -> int:
    return N.load().lbm_work_bytes(ctypes.byref(params))


class Sim:
    """One filtered LB-MHD run on one GPU (names follow the C ABI)."""

    def __init__(self, nx, ny, nu, eta, delta=0.0, closure_scale=1.0, s5=0.0, s6=0.0, s7=0.0, s8=0.0,
                 grad_stencil="iso9", dtype="fp64", schedule="fused", rho0=1.0, b_ref=(0.0, 0.0),
                 closure="analytic", mag_lattice="d2q5", device="cuda:0", stream=None):
        import torch

        lib = N.load()
        self._torch = torch
        self.params = make_params(nx, ny, nu, eta, delta, closure_scale, s5, s6, s7, s8,
                                  grad_stencil, dtype, schedule, rho0, b_ref, closure, mag_lattice)
        self.nx, self.ny = int(nx), int(ny)
        # populations per cell: 9 f plus two components of g on 5 or 9 velocities
        self.npop = 9 + 2 * (9 if mag_lattice == "d2q9" else 5)
        self.device = torch.device(device)
        sb = lib.lbm_state_bytes(ctypes.byref(self.params))
        wb = lib.lbm_work_bytes(ctypes.byref(self.params))
        if sb == 0 or wb == 0:
            # let lbm_create report the exact reason
            ctx = ctypes.c_void_p()
            N.check(lib.lbm_create(ctypes.byref(ctx), ctypes.byref(self.params), None, None, None), "lbm_create")
        self.state_buf = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.work_buf = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        N.check(lib.lbm_create(ctypes.byref(self._ctx), ctypes.byref(self.params),
                               ctypes.c_void_p(self.state_buf.data_ptr()),
                               ctypes.c_void_p(self.work_buf.data_ptr()),
                               ctypes.c_void_p(self.stream.cuda_stream)), "lbm_create")
        self._lib = lib

    # -- the ABI -----------------------------------------------------------
    def init_kh_jet(self, U0=0.05, delta_over_L=0.05, B0=0.01, rho0=1.0, pert_amp_over_U0=1e-3,
                    noise_amp=1e-5, seed=0):
        kh = N.LbmKhParams(U0=U0, delta_over_L=delta_over_L, B0=B0, rho0=rho0,
                           pert_amp_over_U0=pert_amp_over_U0, noise_amp=noise_amp, seed=int(seed))
        N.check(self._lib.lbm_init_kh_jet(self._ctx, ctypes.byref(kh)), "lbm_init_kh_jet")

    def init_sech2_jet(self, U0=4.88e-2, B0=0.005 * 4.88e-2, pert=0.01, k=4, rho0=1.0):
        """The magnetized Kelvin-Helmholtz jet of Sec. 4 (lbm_init_sech2_jet)."""
        jet = N.LbmSech2Params(U0=U0, B0=B0, pert=pert, rho0=rho0, k=int(k), reserved=0)
        N.check(self._lib.lbm_init_sech2_jet(self._ctx, ctypes.byref(jet)), "lbm_init_sech2_jet")

    def init_from_moments(self, mom, t: int = 0):
        """Equilibrium state of given fields mom [5, ny, nx] float64 (rho, m_x,
        m_y, B_x, B_y; any device), time t."""
        m = self._torch.as_tensor(mom, dtype=self._torch.float64).to(self.device).contiguous()
        self._check_field(m, 5)
        N.check(self._lib.lbm_init_from_moments(self._ctx, ctypes.c_void_p(m.data_ptr()), int(t)),
                "lbm_init_from_moments")
        self._keep = m

    def step(self, n: int = 1):
        N.check(self._lib.lbm_step(self._ctx, int(n)), "lbm_step")

    @property
    def t(self) -> int:
        t = ctypes.c_int64()
        N.check(self._lib.lbm_get_time(self._ctx, ctypes.byref(t)), "lbm_get_time")
        return t.value

    def moments(self, out=None):
        """[5, ny, nx] float64 device tensor: rho, m_x, m_y, B_x, B_y."""
        if out is None:
            out = self._torch.empty((5, self.ny, self.nx), dtype=self._torch.float64, device=self.device)
        self._check_field(out, 5)
        N.check(self._lib.lbm_moments(self._ctx, ctypes.c_void_p(out.data_ptr())), "lbm_moments")
        return out

    def get_state(self, out=None):
        """[npop, ny, nx] float64 device tensor of the populations at time t
        (npop = 19 with D2Q5 g, 27 with D2Q9 g)."""
        if out is None:
            out = self._torch.empty((self.npop, self.ny, self.nx), dtype=self._torch.float64, device=self.device)
        self._check_field(out, self.npop)
        N.check(self._lib.lbm_get_state(self._ctx, ctypes.c_void_p(out.data_ptr())), "lbm_get_state")
        return out

    def set_state(self, state, t: int = 0):
        """state: [npop, ny, nx] float64 (any device; copied to this GPU)."""
        s = self._torch.as_tensor(state, dtype=self._torch.float64).to(self.device).contiguous()
        self._check_field(s, self.npop)
        N.check(self._lib.lbm_set_state(self._ctx, ctypes.c_void_p(s.data_ptr()), int(t)), "lbm_set_state")
        self._keep = s  # the copy must outlive the asynchronous kernel

    def diagnostics(self, raise_nonfinite: bool = False) -> dict:
        d = N.LbmDiag()
        rc = self._lib.lbm_diagnostics(self._ctx, ctypes.byref(d))
        if rc != N.LBM_ENONFINITE or raise_nonfinite:
            N.check(rc, "lbm_diagnostics")
        return {name: getattr(d, name) for name, _ in N.LbmDiag._fields_}

    def set_closure_mlp(self, packed):
        """Install a packed network (a uint8 device tensor of LBM_MLP_PACKED_BYTES,
        see learned.Mlp.packed) in a context created with closure="learned"."""
        self._check_buf(packed, N.LBM_MLP_PACKED_BYTES)
        N.check(self._lib.lbm_set_closure_mlp(self._ctx, ctypes.c_void_p(packed.data_ptr())), "lbm_set_closure_mlp")
        self._stream_sync_keep = packed

    def set_correction_interval(self, every: int):
        """Learned closure: evaluate the network every `every` steps (at steps
        t with t % every == 0 and at the first step after a new state or
        network) and hold its correction in between."""
        N.check(self._lib.lbm_set_correction_interval(self._ctx, int(every)), "lbm_set_correction_interval")

    def closure_correction(self, out=None):
        """[4, ny, nx] float32 device tensor: the network's tau_xx, tau_xy, tau_yy,
        eps corrections of the current state."""
        torch = self._torch
        if out is None:
            out = torch.empty((4, self.ny, self.nx), dtype=torch.float32, device=self.device)
        if out.dtype != torch.float32 or tuple(out.shape) != (4, self.ny, self.nx) or not out.is_contiguous() \
                or out.data_ptr() % 256:
            raise ValueError("expected a contiguous aligned float32 tensor of shape (4, ny, nx)")
        N.check(self._lib.lbm_closure_correction(self._ctx, ctypes.c_void_p(out.data_ptr())), "lbm_closure_correction")
        return out

    def _check_buf(self, t, nbytes):
        if t.device != self.device or not t.is_contiguous() or t.numel() * t.element_size() < nbytes \
                or t.data_ptr() % 256:
            raise ValueError(f"expected a contiguous aligned device buffer of >= {nbytes} bytes on {self.device}")

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.lbm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_field(self, t, planes):
        torch = self._torch
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous() \
                or tuple(t.shape) != (planes, self.ny, self.nx):
            raise ValueError(f"expected a contiguous float64 tensor of shape ({planes}, {self.ny}, {self.nx}) "
                             f"on {self.device}")
        if t.data_ptr() % 256:
            raise ValueError("device buffer must be 256-byte aligned")
