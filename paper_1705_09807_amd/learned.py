"""Python front end of include/lbmhd_learned.h: argument marshalling only.

The network's forward and backward passes, the optimiser, the filtered-DNS
pipeline (filter, subsample, closure samples), the normalisation statistics
and the spectra all run in the HIP kernels of liblbmhd.so; torch supplies
device memory and the stream.
"""

from __future__ import annotations

import ctypes
import math

from . import native as N

_STENCILS = {"iso9": N.LBM_STENCIL_ISO9, "central5": N.LBM_STENCIL_CENTRAL5}


def _torch():
    import torch
    return torch


def _ptr(t):
    if t is None:
        return None
    if t.data_ptr() % 256:
        raise ValueError("device buffers must be 256-byte aligned")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream, device):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _contig(t, dtype, shape=None):
    torch = _torch()
    if t.dtype != dtype or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def flat_params(w1, b1, w2, b2, w3, b3):
    """Concatenate (w1 [64|63, 64], b1 [64], w2 [64, 64], b2, w3 [64, 4], b3) into
    the LBM_MLP_PARAMS layout (w1's pad row 63 zero)."""
    torch = _torch()
    w1 = torch.as_tensor(w1, dtype=torch.float32)
    if w1.shape[0] == 63:
        w1 = torch.cat([w1, torch.zeros(1, 64, dtype=torch.float32)])
    parts = [w1.reshape(-1), b1, w2, b2, w3, b3]
    flat = torch.cat([torch.as_tensor(p, dtype=torch.float32).reshape(-1) for p in parts])
    assert flat.numel() == N.LBM_MLP_PARAMS
    return flat


def glorot_params(seed: int):
    """Glorot-uniform weights, zero biases, w1's pad row zero (flat FP32, host)."""
    torch = _torch()
    g = torch.Generator().manual_seed(int(seed))

    def u(fi, fo):
        lim = math.sqrt(6.0 / (fi + fo))
        return (torch.rand(fi, fo, generator=g, dtype=torch.float64) * 2 - 1).mul(lim).float()

    return flat_params(u(63, 64), torch.zeros(64), u(64, 64), torch.zeros(64), u(64, 4), torch.zeros(4))


class Mlp:
    """The closure network on one GPU: FP32 master parameters, Adam moments,
    normalisation and the packed bfloat16 copy the kernels read."""

    def __init__(self, params, device="cuda:0", stream=None):
        torch = _torch()
        self._lib = N.load()
        self.device = torch.device(device)
        self.stream = stream
        self.params = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous().clone()
        if self.params.numel() != N.LBM_MLP_PARAMS:
            raise ValueError(f"expected {N.LBM_MLP_PARAMS} parameters")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = 0
        self.norm = torch.zeros(32, dtype=torch.float32, device=self.device)   # lbm_mlp_norm
        self.norm[8:16] = 1.0
        self.norm[16:20] = 1.0
        self.packed = torch.empty(N.LBM_MLP_PACKED_BYTES, dtype=torch.uint8, device=self.device)
        self.grad = torch.zeros_like(self.params)
        self._work = None

    # -- normalisation -----------------------------------------------------
    def set_norm(self, shift, scale, out_scale):
        """shift, scale: 7 per-field values; out_scale: 4 values."""
        torch = _torch()
        nm = torch.zeros(32, dtype=torch.float32)
        nm[:7] = torch.as_tensor(shift, dtype=torch.float32)[:7]
        nm[8:15] = torch.as_tensor(scale, dtype=torch.float32)[:7]
        nm[15] = 1.0
        nm[16:20] = torch.as_tensor(out_scale, dtype=torch.float32)
        self.norm.copy_(nm.to(self.device))

    def fit_norm(self, X, T):
        """Normalisation from training rows (lbm_mlp_feature_stats)."""
        torch = _torch()
        n = _contig(X, torch.float32).shape[0]
        _contig(T, torch.float32, (n, 4))
        wb = self._lib.lbm_mlp_stats_work_bytes(n)
        work = torch.empty(max(wb, 1), dtype=torch.uint8, device=self.device)
        N.check(self._lib.lbm_mlp_feature_stats(_ptr(X), _ptr(T), n, _ptr(self.norm), _ptr(work), wb,
                                                _stream(self.stream, self.device)), "lbm_mlp_feature_stats")
        self._keep = work

    # -- network -----------------------------------------------------------
    def pack(self):
        N.check(self._lib.lbm_mlp_pack(_ptr(self.params), _ptr(self.norm), _ptr(self.packed),
                                       _stream(self.stream, self.device)), "lbm_mlp_pack")
        return self.packed

    def forward(self, X):
        """(y [n, 4] float32, ood [n] int32) of feature rows X [n, 64] (packs first)."""
        torch = _torch()
        n = _contig(X, torch.float32).shape[0]
        if X.dim() != 2 or X.shape[1] != 64:
            raise ValueError("X must be [n, 64]")
        self.pack()
        y = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        ood = torch.empty(n, dtype=torch.int32, device=self.device)
        N.check(self._lib.lbm_mlp_forward(_ptr(self.packed), _ptr(X), n, _ptr(y), _ptr(ood),
                                          _stream(self.stream, self.device)), "lbm_mlp_forward")
        return y, ood

    def _train_work(self, batch):
        torch = _torch()
        wb = self._lib.lbm_mlp_train_work_bytes(int(batch))
        if wb == 0:
            raise ValueError("batch must lie in [1, 2^20]")
        if self._work is None or self._work.numel() < wb:
            self._work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        return wb

    def gradient(self, X, T, idx):
        """Batch gradient (into self.grad) and loss (1-element tensor) over rows idx."""
        torch = _torch()
        batch = _contig(idx, torch.int32).numel()
        wb = self._train_work(batch)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        N.check(self._lib.lbm_mlp_gradient(_ptr(self.params), _ptr(self.norm), _ptr(X), _ptr(T), _ptr(idx), batch,
                                           _ptr(self._work), wb, _ptr(self.grad), _ptr(loss),
                                           _stream(self.stream, self.device)), "lbm_mlp_gradient")
        return self.grad, loss

    def adam(self, grad, lr: float):
        self.step_count += 1
        N.check(self._lib.lbm_mlp_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(grad),
                                       self.step_count, float(lr), _stream(self.stream, self.device)),
                "lbm_mlp_adam")

    def train_step(self, X, T, idx, lr: float):
        """One Adam step on rows idx of (X, T); returns the batch loss (device)."""
        torch = _torch()
        batch = _contig(idx, torch.int32).numel()
        _contig(X, torch.float32)
        _contig(T, torch.float32)
        wb = self._train_work(batch)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        self.step_count += 1
        N.check(self._lib.lbm_mlp_train_step(_ptr(self.params), _ptr(self.m), _ptr(self.v), self.step_count,
                                             float(lr), _ptr(self.norm), _ptr(X), _ptr(T), _ptr(idx), batch,
                                             _ptr(self._work), wb, _ptr(loss), _stream(self.stream, self.device)),
                "lbm_mlp_train_step")
        return loss


def filter_subsample(mom, factor: int, delta: float, stream=None):
    """[12, ny/f, nx/f] float64: the Gaussian-filtered, subsampled fields and
    products of the moments mom [5, ny, nx] (float64 device tensor)."""
    torch = _torch()
    lib = N.load()
    _contig(mom, torch.float64)
    _, ny, nx = mom.shape
    wb = lib.lbm_filter_work_bytes(nx, ny, int(factor), float(delta))
    if wb == 0:
        raise ValueError("invalid filter arguments")
    work = torch.empty(wb, dtype=torch.uint8, device=mom.device)
    out = torch.empty((12, ny // factor, nx // factor), dtype=torch.float64, device=mom.device)
    N.check(lib.lbm_filter_subsample(_ptr(mom), nx, ny, int(factor), float(delta), _ptr(out), _ptr(work), wb,
                                     _stream(stream, mom.device)), "lbm_filter_subsample")
    torch.cuda.current_stream(mom.device).synchronize() if stream is None else stream.synchronize()
    return out


def closure_samples(coarse, delta: float, stencil="iso9", stream=None):
    """(X [n, 64] float32, T [n, 4] float32) of every cell of the filtered
    coarse fields coarse [12, ny, nx] (float64 device tensor)."""
    torch = _torch()
    lib = N.load()
    _contig(coarse, torch.float64)
    _, ny, nx = coarse.shape
    X = torch.empty((nx * ny, 64), dtype=torch.float32, device=coarse.device)
    T = torch.empty((nx * ny, 4), dtype=torch.float32, device=coarse.device)
    N.check(lib.lbm_closure_samples(_ptr(coarse), nx, ny, float(delta), _STENCILS[stencil], _ptr(X), _ptr(T),
                                    _stream(stream, coarse.device)), "lbm_closure_samples")
    return X, T


def spectra(mom, stream=None):
    """(E_K [nbins], E_M [nbins], E_x [n/2+1]) float64 of moments mom [5, n, n]."""
    torch = _torch()
    lib = N.load()
    _contig(mom, torch.float64)
    n = mom.shape[1]
    if mom.shape[2] != n:
        raise ValueError("spectra need a square grid")
    nb = lib.lbm_spectra_bins(n)
    wb = lib.lbm_spectra_work_bytes(n)
    if nb == 0 or wb == 0:
        raise ValueError("n must be a power of two in [8, 16384]")
    work = torch.empty(wb, dtype=torch.uint8, device=mom.device)
    ek = torch.empty(nb, dtype=torch.float64, device=mom.device)
    em = torch.empty(nb, dtype=torch.float64, device=mom.device)
    ekx = torch.empty(n // 2 + 1, dtype=torch.float64, device=mom.device)
    N.check(lib.lbm_spectra(_ptr(mom), n, _ptr(ek), _ptr(em), _ptr(ekx), _ptr(work), wb,
                            _stream(stream, mom.device)), "lbm_spectra")
    torch.cuda.current_stream(mom.device).synchronize() if stream is None else stream.synchronize()
    return ek, em, ekx
