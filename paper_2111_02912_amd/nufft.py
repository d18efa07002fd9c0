"""Torch-facing wrapper of the C ABI: one plan per image shape.

All arithmetic runs in the HIP library; this module checks tensor
arguments, allocates outputs with PyTorch and passes device pointers and the
current HIP stream through ctypes.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import check


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class TorchAllocator:
    """kbn_allocator backed by PyTorch's caching allocator: every device
    buffer of a plan is a uint8 tensor, so plan memory shows in
    torch.cuda.memory_allocated and is reused by PyTorch after the plan frees
    it.  A block is allocated on the stream the library names; a block
    released on another stream is marked with record_stream, so PyTorch does
    not hand it out again before that stream's queued work has run."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.live = {}  # data pointer -> (tensor, stream handle of the allocation)
        self.calls = [0, 0]  # allocations, releases
        self._alloc_cb = _lib.ALLOC_FN(self._alloc)
        self._free_cb = _lib.FREE_FN(self._free)
        self.struct = _lib.KbnAllocator(None, self._alloc_cb, self._free_cb)

    def _torch_stream(self, handle):
        if not handle:
            return torch.cuda.default_stream(self.device)
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream == handle:
            return cur
        return torch.cuda.ExternalStream(handle, device=self.device)

    def _alloc(self, ctx, nbytes, stream):
        try:
            with torch.cuda.stream(self._torch_stream(stream)):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:  # out of memory (or any failure): the library reports KBN_ERR_OOM
            return None
        self.calls[0] += 1
        self.live[t.data_ptr()] = (t, stream or 0)
        return t.data_ptr()

    def _free(self, ctx, ptr, stream):
        t, s0 = self.live.pop(ptr, (None, 0))
        if t is None:
            return
        self.calls[1] += 1
        try:
            if (stream or 0) != s0:
                t.record_stream(self._torch_stream(stream))
        except Exception:
            pass
        del t

    @property
    def live_bytes(self) -> int:
        return sum(t.numel() for t, _ in self.live.values())


def footprint(N: Sequence[int], M: int, B: int = 1, C: int = 1, jac: bool = False, sigma: float = 2.0,
              J: int = 6, max_workspace: int = 0, accuracy: Optional[str] = None) -> int:
    """Device bytes of a plan for images N with M points and calls of B
    images x C coils (kbn_plan_footprint; host-only, no GPU needed)."""
    if accuracy is not None:
        sigma, J = ACCURACY[accuracy]
    opts = _lib.KbnOpts()
    opts.sigma = float(sigma)
    opts.J = int(J)
    opts.max_workspace = int(max_workspace)
    N = tuple(int(n) for n in N)
    arr = (ctypes.c_int64 * len(N))(*N)
    out = ctypes.c_int64()
    check(_lib.lib().kbn_plan_footprint(len(N), arr, ctypes.byref(opts), int(M), int(B), int(C), int(bool(jac)),
                                        ctypes.byref(out)), "kbn_plan_footprint")
    return out.value


# (sigma, J) presets: the default high-accuracy setting (relative error
# ~7e-6 against the NUDFT) and the low-accuracy setting used for training
# in Sec. IV-C (grid 1.25 N, J = 5; error ~1e-3)
ACCURACY = {"high": (2.0, 6), "low": (1.25, 5)}


class KbNufft:
    """Kaiser-Bessel NUFFT plan for images of shape ``N`` on one GPU.

    Shapes: omega [M, D] float32; images [B, *N] complex64; coil maps
    [C, *N] complex64; k-space [B, C, M] complex64.
    """

    def __init__(self, N: Sequence[int], sigma: float = 2.0, J: int = 6,
                 tile: Optional[Sequence[int]] = None, max_workspace: int = 0,
                 spread_tile: int = 0, device=None, accuracy: Optional[str] = None,
                 allocator: Optional[TorchAllocator] = None):
        if accuracy is not None:
            if accuracy not in ACCURACY:
                raise ValueError(f"accuracy must be one of {sorted(ACCURACY)}, got {accuracy!r}")
            sigma, J = ACCURACY[accuracy]
        self.N = tuple(int(n) for n in N)
        self.D = len(self.N)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        L = _lib.lib()
        opts = _lib.KbnOpts()
        opts.sigma = float(sigma)
        opts.J = int(J)
        if tile is not None:
            for d, t in enumerate(tile):
                opts.tile[d] = int(t)
        opts.max_workspace = int(max_workspace)
        opts.spread_tile = int(spread_tile)
        self.opts = {"sigma": float(sigma), "J": int(J), "tile": tuple(tile) if tile else None,
                     "spread_tile": int(spread_tile)}
        arr = (ctypes.c_int64 * self.D)(*self.N)
        h = ctypes.c_void_p()
        self.allocator = allocator if allocator is not None else TorchAllocator(self.device)
        with torch.cuda.device(self.device):
            check(L.kbn_plan_create(ctypes.byref(h), self.D, arr, ctypes.byref(opts),
                                    ctypes.byref(self.allocator.struct), _stream(self.device)),
                  "kbn_plan_create")
        self._h = h
        self.M = None
        info = self.info()
        self.K = info["K"]
        self.beta = info["beta"]
        self.tile = info["tile"]
        self.ntiles = info["ntiles"]

    # -- lifecycle -------------------------------------------------------
    def close(self):
        """Release the plan; its memory goes back to PyTorch in stream order
        on the current stream."""
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().kbn_plan_destroy(self._h, _stream(self.device))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks ---------------------------------------------------
    def _img(self, x: torch.Tensor, name: str) -> torch.Tensor:
        if x.dtype != torch.complex64 or x.device != self.device:
            raise TypeError(f"{name} must be complex64 on {self.device}")
        if tuple(x.shape[-self.D:]) != self.N:
            raise ValueError(f"{name} trailing shape {tuple(x.shape[-self.D:])} != {self.N}")
        return x.reshape((-1,) + self.N).contiguous()

    def _ksp(self, y: torch.Tensor, B: int, C: int, name: str) -> torch.Tensor:
        if y.dtype != torch.complex64 or y.device != self.device:
            raise TypeError(f"{name} must be complex64 on {self.device}")
        if y.numel() != B * C * self.M:
            raise ValueError(f"{name} has {y.numel()} elements, expected B*C*M = {B * C * self.M}")
        return y.reshape(B, C, self.M).contiguous()

    def _maps(self, smaps):
        if smaps is None:
            return None, 1
        s = self._img(smaps, "smaps")
        return s, s.shape[0]

    def _need_points(self):
        if self.M is None:
            raise RuntimeError("set_points() has not been called")

    # -- C ABI calls -------------------------------------------------------
    def set_points(self, omega: torch.Tensor):
        if omega.dtype != torch.float32 or omega.device != self.device or omega.dim() != 2 \
                or omega.shape[1] != self.D:
            raise TypeError(f"omega must be float32 [M, {self.D}] on {self.device}")
        om = omega.contiguous()
        check(_lib.lib().kbn_set_points(self._h, om.shape[0], _ptr(om), _stream(self.device)),
              "kbn_set_points")
        self.M = int(om.shape[0])
        self._omega_keep = om  # keep alive until the stream has consumed it
        self._points_src = omega
        self._points_key = self._omega_key(omega)
        return self

    @staticmethod
    def _omega_key(omega: torch.Tensor):
        return (omega.data_ptr(), omega._version, tuple(omega.shape), tuple(omega.stride()))

    def ensure_points(self, omega: torch.Tensor):
        """set_points(omega) unless this plan's points came from the same,
        unmodified tensor (the plan keeps a reference to it, so its memory
        cannot be recycled while the key is held)."""
        if self.M is None or getattr(self, "_points_src", None) is None \
                or self._points_key != self._omega_key(omega):
            self.set_points(omega.detach())
            self._points_src = omega
            self._points_key = self._omega_key(omega)
        return self

    def forward(self, x: torch.Tensor, smaps: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y[b, c] = A(omega)(s_c * x_b); returns [B, C, M]."""
        self._need_points()
        xx = self._img(x, "x")
        s, C = self._maps(smaps)
        B = xx.shape[0]
        y = torch.empty((B, C, self.M), dtype=torch.complex64, device=self.device)
        check(_lib.lib().kbn_forward(self._h, B, C, _ptr(xx), _ptr(s), _ptr(y), _stream(self.device)),
              "kbn_forward")
        return y

    def adjoint(self, y: torch.Tensor, smaps: Optional[torch.Tensor] = None) -> torch.Tensor:
        """x_b = sum_c conj(s_c) A(omega)^H y[b, c]; y [B, C, M] -> [B, *N]."""
        self._need_points()
        s, C = self._maps(smaps)
        B = y.numel() // (C * self.M) if self.M else y.shape[0]
        yy = self._ksp(y, B, C, "y")
        x = torch.empty((B,) + self.N, dtype=torch.complex64, device=self.device)
        check(_lib.lib().kbn_adjoint(self._h, B, C, _ptr(yy), _ptr(s), _ptr(x), _stream(self.device)),
              "kbn_adjoint")
        return x

    def jac_omega_fwd(self, x: torch.Tensor, g: torch.Tensor, smaps=None, out=None,
                      accumulate: bool = False) -> torch.Tensor:
        """dL/domega for y = E x given g = dL/dy; returns [M, D] float32."""
        self._need_points()
        xx = self._img(x, "x")
        s, C = self._maps(smaps)
        B = xx.shape[0]
        gg = self._ksp(g, B, C, "g")
        dom = out if out is not None else torch.empty((self.M, self.D), dtype=torch.float32, device=self.device)
        check(_lib.lib().kbn_jac_omega_fwd(self._h, B, C, _ptr(xx), _ptr(s), _ptr(gg), _ptr(dom),
                                           int(accumulate), _stream(self.device)), "kbn_jac_omega_fwd")
        return dom

    def forward_jac_omega(self, x: torch.Tensor, g: torch.Tensor, smaps=None, out=None,
                          accumulate: bool = False):
        """forward(x) and jac_omega_fwd(x, g) in one library call (g known
        before y); returns (y [B, C, M], dL/domega [M, D] float32)."""
        self._need_points()
        xx = self._img(x, "x")
        s, C = self._maps(smaps)
        B = xx.shape[0]
        gg = self._ksp(g, B, C, "g")
        y = torch.empty((B, C, self.M), dtype=torch.complex64, device=self.device)
        dom = out if out is not None else torch.empty((self.M, self.D), dtype=torch.float32, device=self.device)
        check(_lib.lib().kbn_forward_jac_omega(self._h, B, C, _ptr(xx), _ptr(s), _ptr(y), _ptr(gg), _ptr(dom),
                                               int(accumulate), _stream(self.device)), "kbn_forward_jac_omega")
        return y, dom

    def jac_omega_adj(self, y: torch.Tensor, g: torch.Tensor, smaps=None, out=None,
                      accumulate: bool = False) -> torch.Tensor:
        """dL/domega for x = E^H y given g = dL/dx; returns [M, D] float32."""
        self._need_points()
        gg = self._img(g, "g")
        s, C = self._maps(smaps)
        B = gg.shape[0]
        yy = self._ksp(y, B, C, "y")
        dom = out if out is not None else torch.empty((self.M, self.D), dtype=torch.float32, device=self.device)
        check(_lib.lib().kbn_jac_omega_adj(self._h, B, C, _ptr(yy), _ptr(s), _ptr(gg), _ptr(dom),
                                           int(accumulate), _stream(self.device)), "kbn_jac_omega_adj")
        return dom

    def jac_x(self, op: int, g: torch.Tensor, smaps=None) -> torch.Tensor:
        """Gradient w.r.t. the linear input: E^H g (op FORWARD) or E g (op ADJOINT)."""
        self._need_points()
        s, C = self._maps(smaps)
        if op == _lib.KBN_OP_FORWARD:
            B = g.numel() // (C * self.M)
            gg = self._ksp(g, B, C, "g")
            out = torch.empty((B,) + self.N, dtype=torch.complex64, device=self.device)
        elif op == _lib.KBN_OP_ADJOINT:
            gg = self._img(g, "g")
            B = gg.shape[0]
            out = torch.empty((B, C, self.M), dtype=torch.complex64, device=self.device)
        else:
            raise ValueError("op must be KBN_OP_FORWARD or KBN_OP_ADJOINT")
        check(_lib.lib().kbn_jac_x(self._h, op, B, C, _ptr(gg), _ptr(s), _ptr(out), _stream(self.device)),
              "kbn_jac_x")
        return out

    # -- off-resonance model (Sec. II-H): E = sum_l diag(b_l) A diag(c_l) S --
    def _seg(self, b: torch.Tensor, c: torch.Tensor):
        if c.dtype != torch.complex64 or c.device != self.device or c.dim() != self.D + 1 \
                or tuple(c.shape[1:]) != self.N:
            raise TypeError(f"c must be complex64 [L, *{self.N}] on {self.device}")
        L = int(c.shape[0])
        if b.dtype != torch.complex64 or b.device != self.device or tuple(b.shape) != (L, self.M):
            raise TypeError(f"b must be complex64 [{L}, {self.M}] on {self.device}")
        return b.contiguous(), c.contiguous(), L

    def field_forward(self, x, b, c, smaps=None) -> torch.Tensor:
        """y[b, k] = sum_l b_l (.) A(c_l s_k x_b); returns [B, C, M]."""
        self._need_points()
        xx = self._img(x, "x")
        s, C = self._maps(smaps)
        bb, cc, L = self._seg(b, c)
        B = xx.shape[0]
        y = torch.empty((B, C, self.M), dtype=torch.complex64, device=self.device)
        check(_lib.lib().kbn_field_forward(self._h, B, C, L, _ptr(xx), _ptr(s), _ptr(bb), _ptr(cc), _ptr(y),
                                           _stream(self.device)), "kbn_field_forward")
        return y

    def field_adjoint(self, y, b, c, smaps=None) -> torch.Tensor:
        """x_b = sum_{l,k} conj(c_l s_k) (.) A^H(conj(b_l) (.) y[b, k]); [B, *N]."""
        self._need_points()
        s, C = self._maps(smaps)
        bb, cc, L = self._seg(b, c)
        B = y.numel() // (C * self.M) if self.M else y.shape[0]
        yy = self._ksp(y, B, C, "y")
        x = torch.empty((B,) + self.N, dtype=torch.complex64, device=self.device)
        check(_lib.lib().kbn_field_adjoint(self._h, B, C, L, _ptr(yy), _ptr(s), _ptr(bb), _ptr(cc), _ptr(x),
                                           _stream(self.device)), "kbn_field_adjoint")
        return x

    def field_jac_omega_fwd(self, x, g, b, c, smaps=None, out=None, accumulate: bool = False):
        """dL/domega for y = E_f x given g = dL/dy [B, C, M]; returns [M, D]."""
        self._need_points()
        xx = self._img(x, "x")
        s, C = self._maps(smaps)
        bb, cc, L = self._seg(b, c)
        B = xx.shape[0]
        gg = self._ksp(g, B, C, "g")
        dom = out if out is not None else torch.empty((self.M, self.D), dtype=torch.float32, device=self.device)
        check(_lib.lib().kbn_field_jac_omega_fwd(self._h, B, C, L, _ptr(xx), _ptr(s), _ptr(bb), _ptr(cc),
                                                 _ptr(gg), _ptr(dom), int(accumulate), _stream(self.device)),
              "kbn_field_jac_omega_fwd")
        return dom

    def field_jac_omega_adj(self, y, g, b, c, smaps=None, out=None, accumulate: bool = False):
        """dL/domega for x = E_f^H y given g = dL/dx [B, *N]; returns [M, D]."""
        self._need_points()
        gg = self._img(g, "g")
        s, C = self._maps(smaps)
        bb, cc, L = self._seg(b, c)
        B = gg.shape[0]
        yy = self._ksp(y, B, C, "y")
        dom = out if out is not None else torch.empty((self.M, self.D), dtype=torch.float32, device=self.device)
        check(_lib.lib().kbn_field_jac_omega_adj(self._h, B, C, L, _ptr(yy), _ptr(s), _ptr(bb), _ptr(cc),
                                                 _ptr(gg), _ptr(dom), int(accumulate), _stream(self.device)),
              "kbn_field_jac_omega_adj")
        return dom

    def field_segments(self, t: torch.Tensor, w: torch.Tensor, L: int, t0=None, t1=None):
        """Linear-interpolation time segmentation (b [L, M], c [L, *N]) for
        readout times t [M] (s) and field map w [*N] (rad/s); the segment
        times span [t0, t1] (default: the range of t)."""
        if t.dtype != torch.float32 or t.device != self.device or t.dim() != 1:
            raise TypeError(f"t must be float32 [M] on {self.device}")
        if w.dtype != torch.float32 or w.device != self.device or tuple(w.shape) != self.N:
            raise TypeError(f"w must be float32 {self.N} on {self.device}")
        M = int(t.shape[0])
        if t0 is None or t1 is None:
            lo, hi = (float(t.min()), float(t.max())) if M else (0.0, 0.0)
            t0 = lo if t0 is None else t0
            t1 = hi if t1 is None else t1
        b = torch.empty((int(L), M), dtype=torch.complex64, device=self.device)
        c = torch.empty((int(L),) + self.N, dtype=torch.complex64, device=self.device)
        tt, ww = t.contiguous(), w.contiguous()
        npix = 1
        for n in self.N:
            npix *= n
        check(_lib.lib().kbn_field_segments(M, _ptr(tt), float(t0), float(t1), npix, _ptr(ww), int(L),
                                            _ptr(b), _ptr(c), _stream(self.device)), "kbn_field_segments")
        return b, c

    def info(self) -> dict:
        K = (ctypes.c_int64 * 3)()
        T = (ctypes.c_int * 3)()
        nt = ctypes.c_int()
        beta = ctypes.c_double()
        M = ctypes.c_int64()
        ws = ctypes.c_int64()
        db = ctypes.c_int64()
        check(_lib.lib().kbn_plan_info(self._h, K, T, ctypes.byref(nt), ctypes.byref(beta),
                                       ctypes.byref(M), ctypes.byref(ws), ctypes.byref(db)), "kbn_plan_info")
        return {"K": tuple(K[d] for d in range(self.D)), "tile": tuple(T[d] for d in range(self.D)),
                "ntiles": nt.value, "beta": beta.value, "M": M.value, "workspace_bytes": ws.value,
                "device_bytes": db.value}

    def get_points(self) -> dict:
        """Index pass results: sorted order, cells, fractions, tile offsets."""
        self._need_points()
        M, D = self.M, self.D
        dev = self.device
        order = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
        cell = torch.empty((D, max(M, 1)), dtype=torch.int32, device=dev)
        frac = torch.empty((D, max(M, 1)), dtype=torch.float32, device=dev)
        off = torch.empty(self.ntiles + 2, dtype=torch.int32, device=dev)
        check(_lib.lib().kbn_get_points(self._h, _ptr(order), _ptr(cell), _ptr(frac), _ptr(off),
                                        _stream(self.device)), "kbn_get_points")
        return {"order": order[:M], "cell": cell[:, :M], "frac": frac[:, :M], "offsets": off}

    def timing(self, enable: bool, classes=None):
        """Start (clearing counters) or stop per-kernel event timing;
        `classes` (names, default all) limits the events to those kernel
        classes."""
        if enable:
            mask = 0xFFFFFFFF
            if classes is not None:
                names = self.timing_classes()
                mask = 0
                for c in classes:
                    mask |= 1 << names.index(c)
            check(_lib.lib().kbn_timing_select(self._h, mask), "kbn_timing_select")
        check(_lib.lib().kbn_timing(self._h, int(bool(enable))), "kbn_timing")

    @staticmethod
    def timing_classes():
        """Kernel class names in class order."""
        L = _lib.lib()
        out = []
        while True:
            name = L.kbn_timing_name(len(out))
            if name is None:
                return out
            out.append(name.decode())

    def timing_read(self) -> dict:
        """{class name: (launches, total ms)} of the timed launches so far."""
        L = _lib.lib()
        out = {}
        c = 0
        while True:
            name = L.kbn_timing_name(c)
            if name is None:
                break
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            check(L.kbn_timing_read(self._h, c, ctypes.byref(n), ctypes.byref(ms)), "kbn_timing_read")
            out[name.decode()] = (n.value, ms.value)
            c += 1
        return out

    def check_error(self) -> int:
        """Synchronise and return the sticky non-finite flag (0 or KBN_ERR_NONFINITE)."""
        rc = _lib.lib().kbn_check_error(self._h, _stream(self.device))
        if rc not in (_lib.KBN_OK, _lib.KBN_ERR_NONFINITE):
            check(rc, "kbn_check_error")
        return rc
