"""ctypes binding of the C ABI in include/recon.h (argument marshalling only).

Every step of the reconstruction runs in the HIP library; this module only
checks shapes and dtypes, passes device pointers and the current HIP stream,
and turns return codes into exceptions.  PyTorch provides device memory and
the stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "librecon.so"

RECON_OK, RECON_NOTCONVERGED, RECON_RESTARTED = 0, 1, 2
RECON_EINVAL, RECON_ENOMEM, RECON_EDEVICE, RECON_ESTATE, RECON_EDIVERGED = -1, -2, -3, -4, -5
GAL, RAN = 0, 1
START_PLAIN, START_FFTA1, START_FFTA2, START_LEARNED = 0, 1, 2, 3
NO_RANDOMS, KEEP_DELTA, START_BUFFERS, CNN_BUFFERS, CNN_HALF, PASS_GRAPHS, LOGNORMAL = 1, 2, 4, 8, 16, 32, 64
FFT_SPLITBF16, FFT_SPLITBF16_X3 = 128, 256
CNN_QUARTER = 512
RELAXED = 1024
CNN_PARAMS = 10833
PAINT_ACCUMULATE, PAINT_NGP = 1, 2
SHIFT_AS_PAINTED = 256

EXPORTED = ("recon_workspace_bytes", "recon_plan", "recon_paint", "recon_solve", "recon_iterate",
            "recon_shift", "recon_get_psi", "recon_get_grid", "recon_get_delta", "recon_set_delta",
            "recon_destroy", "recon_strerror", "recon_last_error", "recon_profile_start",
            "recon_profile_stop", "recon_profile_kernel_name", "recon_cnn_forward", "recon_cnn_train_step",
            "recon_get_radial", "recon_restrict", "recon_prolong", "recon_radial_ratio", "recon_helmholtz",
            "recon_start_restarts", "recon_plan_noalloc", "recon_noalloc_limit", "recon_debug_violations",
            "recon_tile_counts")


class ReconError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"recon error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("batch", ctypes.c_int32), ("box_len", ctypes.c_double),
                ("box_origin", ctypes.c_double * 3), ("observer", ctypes.c_double * 3),
                ("bias", ctypes.c_double), ("growth", ctypes.c_double), ("smooth_r", ctypes.c_double),
                ("mask_tau", ctypes.c_double), ("flags", ctypes.c_uint32), ("max_objects", ctypes.c_int64)]


_LIB = None


def lib_path():
    return os.path.join(_HERE, LIB_NAME)


def debug_lib_path():
    """The library built with the device bounds checks (RECON_DEBUG)."""
    return os.path.join(_HERE, "librecon_debug.so")


def load(path=None):
    """Load the built HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or lib_path()
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is missing; build it with __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, i64, i32, u32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    lib.recon_workspace_bytes.argtypes = [ctypes.POINTER(Params)]
    lib.recon_workspace_bytes.restype = ctypes.c_size_t
    lib.recon_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), vp, ctypes.c_size_t, vp]
    lib.recon_plan_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), vp]
    lib.recon_plan_noalloc.restype = ctypes.c_int
    lib.recon_noalloc_limit.argtypes = []
    lib.recon_noalloc_limit.restype = ctypes.c_size_t
    lib.recon_debug_violations.argtypes = [ctypes.c_int]
    lib.recon_debug_violations.restype = ctypes.c_int64
    lib.recon_paint.argtypes = [vp, ctypes.c_int, vp, vp, i64, vp, u32]
    lib.recon_solve.argtypes = [vp, ctypes.c_int, vp]
    lib.recon_iterate.argtypes = [vp, ctypes.c_int, dbl, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    lib.recon_start_restarts.argtypes = [vp, ctypes.POINTER(i32)]
    lib.recon_tile_counts.argtypes = [vp, ctypes.POINTER(i64)]
    lib.recon_shift.argtypes = [vp, ctypes.c_int, vp, i64, vp, vp, vp]
    lib.recon_get_psi.argtypes = [vp, vp]
    lib.recon_get_grid.argtypes = [vp, ctypes.c_int, vp]
    lib.recon_get_delta.argtypes = [vp, vp]
    lib.recon_set_delta.argtypes = [vp, vp]
    lib.recon_destroy.argtypes = [vp]
    lib.recon_destroy.restype = None
    lib.recon_strerror.argtypes = [ctypes.c_int]
    lib.recon_strerror.restype = ctypes.c_char_p
    lib.recon_last_error.argtypes = [vp]
    lib.recon_last_error.restype = ctypes.c_char_p
    lib.recon_cnn_forward.argtypes = [vp, vp, vp, vp, vp]
    lib.recon_cnn_train_step.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, vp, vp, vp,
                                         ctypes.POINTER(dbl), vp]
    lib.recon_get_radial.argtypes = [vp, vp]
    lib.recon_restrict.argtypes = [vp, vp, vp]
    lib.recon_radial_ratio.argtypes = [vp, vp, dbl, dbl, ctypes.POINTER(dbl)]
    lib.recon_helmholtz.argtypes = [vp, vp, vp, vp]
    lib.recon_prolong.argtypes = [vp, vp, vp]
    lib.recon_profile_start.argtypes = [vp]
    lib.recon_profile_stop.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.c_int]
    lib.recon_profile_kernel_name.argtypes = [ctypes.c_int]
    lib.recon_profile_kernel_name.restype = ctypes.c_char_p
    for name in ("recon_start_restarts", "recon_tile_counts", "recon_cnn_forward", "recon_cnn_train_step", "recon_get_radial", "recon_restrict", "recon_prolong",
                 "recon_radial_ratio", "recon_helmholtz",
                 "recon_profile_start", "recon_profile_stop", "recon_plan", "recon_paint", "recon_solve", "recon_iterate", "recon_shift",
                 "recon_get_psi", "recon_get_grid", "recon_get_delta", "recon_set_delta"):
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _LIB = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_dev(t, dtype, shape_tail, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} must live on {device}")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {shape_tail}]")


class Plan:
    """A reconstruction plan: workspace, geometry, and the C-ABI calls on the current stream."""

    def __init__(self, n, box_len, observer, bias, growth, smooth_r, origin=(0.0, 0.0, 0.0), batch=1,
                 mask_tau=0.1, randoms=True, keep_delta=False, start_buffers=False, max_objects=0, cnn=False,
                 cnn_half=False, graphs=False, lognormal=False, device=None, noalloc=False, split_terms=0,
                 cnn_quarter=False, relaxed=False, lib=None):
        """noalloc=True: the plan runs on the library's own device scratch (recon_plan_noalloc) instead of a
        workspace allocated here; a later no-allocation plan on the same device makes this one stale."""
        self.lib = load() if lib is None else lib    # lib: another build of the library, from load(path)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        flags = (0 if randoms else NO_RANDOMS) | (KEEP_DELTA if keep_delta else 0) | \
                (START_BUFFERS if start_buffers else 0) | (CNN_BUFFERS if cnn else 0) | (CNN_HALF if cnn_half else 0) | \
                (PASS_GRAPHS if graphs else 0) | (LOGNORMAL if lognormal else 0) | \
                {0: 0, 2: FFT_SPLITBF16, 3: FFT_SPLITBF16_X3}[int(split_terms)] | (CNN_QUARTER if cnn_quarter else 0) | \
                (RELAXED if relaxed else 0)
        p = Params()
        p.n, p.batch, p.box_len = int(n), int(batch), float(box_len)
        for a in range(3):
            p.box_origin[a] = float(origin[a])
            p.observer[a] = float(observer[a])
        p.bias, p.growth, p.smooth_r, p.mask_tau, p.flags = float(bias), float(growth), float(smooth_r), \
            float(mask_tau), flags
        p.max_objects = int(max_objects)
        self.params = p
        self.n, self.batch, self.randoms = int(n), int(batch), randoms
        # the catalogue painted last through the brick-binned deposit: (which, pos, pos version, offsets,
        # offsets version).  The plan keeps the tensors alive, so their memory cannot be handed to
        # another tensor while the record stands, and the version counters catch in-place changes.
        self._painted = None
        self.cnn_n = self.n // 4 if cnn_quarter else (self.n // 2 if cnn_half else self.n)     # network grid
        nbytes = self.lib.recon_workspace_bytes(ctypes.byref(p))
        if nbytes == 0:
            raise ReconError(RECON_EINVAL, "invalid parameters")
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        if noalloc:
            self.workspace = None
            with torch.cuda.device(self.device):
                rc = self.lib.recon_plan_noalloc(ctypes.byref(h), ctypes.byref(p),
                                                 ctypes.c_void_p(self.stream.cuda_stream))
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            rc = self.lib.recon_plan(ctypes.byref(h), ctypes.byref(p), _ptr(self.workspace), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream))
        if rc != RECON_OK:
            raise ReconError(rc, self.lib.recon_strerror(rc).decode())
        self.handle = h

    def close(self):
        self._painted = None
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            self.lib.recon_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc, allow=(RECON_OK,)):
        if rc in allow:
            return rc
        msg = self.lib.recon_last_error(self.handle).decode()
        raise ReconError(rc, msg or self.lib.recon_strerror(rc).decode())

    def _check_offsets(self, offsets, n):
        if offsets is None:
            if self.batch > 1 and n > 0:
                raise ValueError("offsets are required when batch > 1")
            return
        _check_dev(offsets, torch.int64, None, "offsets", self.device)
        if offsets.numel() != self.batch + 1:
            raise ValueError("offsets must have batch + 1 entries")

    def paint(self, which, pos, w=None, offsets=None, accumulate=False, ngp=False):
        if which not in (GAL, RAN):
            raise ValueError("which must be GAL or RAN")
        _check_dev(pos, torch.float32, (3,), "pos", self.device)
        if w is not None:
            _check_dev(w, torch.float32, None, "w", self.device)
            if w.numel() != pos.shape[0]:
                raise ValueError("w must have one entry per object")
        self._check_offsets(offsets, pos.shape[0])
        n = pos.shape[0]
        binned = n > 0 and not ngp and n <= self.params.max_objects
        if binned:
            self._painted = None       # the library drops its brick-ordered copy first
        rc = self._rc(self.lib.recon_paint(self.handle, which, _ptr(pos), _ptr(w), n, _ptr(offsets),
                                           (PAINT_ACCUMULATE if accumulate else 0) | (PAINT_NGP if ngp else 0)))
        if binned:
            self._painted = (which, pos, pos._version, offsets, None if offsets is None else offsets._version)
        return rc

    def _as_painted(self, which, pos, offsets):
        # the brick-ordered copy may stand in for pos only when pos is the very tensor painted last,
        # unchanged since (same object, same version), with the same offsets tensor
        rec = self._painted
        if rec is None:
            return False
        w0, p0, v0, o0, ov0 = rec
        return (which == w0 and pos is p0 and pos._version == v0 and offsets is o0
                and (offsets is None or offsets._version == ov0))

    def radial_ratio(self, psi_ref, lo=-1.0, hi=3.0):
        """Table 1 statistic per realisation: (mean, std, outlier fraction, kept count) of
        (psi_ref . r) / (Psi . r); psi_ref [batch, 3, n, n, n] on the device."""
        _check_dev(psi_ref, torch.float32, None, "psi_ref", self.device)
        if psi_ref.numel() != self.batch * 3 * self.n ** 3:
            raise ValueError("psi_ref must hold batch * 3 * n^3 values")
        out = (ctypes.c_double * (4 * self.batch))()
        self._rc(self.lib.recon_radial_ratio(self.handle, _ptr(psi_ref), float(lo), float(hi), out))
        return [tuple(out[4 * b + k] for k in range(4)) for b in range(self.batch)]

    def helmholtz(self, psi_x):
        """Sec. 4.1 split of (psi_x) x: (irrotational, solenoidal), each [batch, 3, n, n, n].
        Resets the plan (paint or set_delta and solve again afterwards)."""
        _check_dev(psi_x, torch.float32, None, "psi_x", self.device)
        if psi_x.numel() != self.batch * self.n ** 3:
            raise ValueError("psi_x must hold batch * n^3 values")
        shape = (self.batch, 3, self.n, self.n, self.n)
        irr = torch.empty(shape, dtype=torch.float32, device=self.device)
        sol = torch.empty(shape, dtype=torch.float32, device=self.device)
        self._rc(self.lib.recon_helmholtz(self.handle, _ptr(psi_x), _ptr(irr), _ptr(sol)))
        return irr, sol

    def set_delta(self, delta):
        _check_dev(delta, torch.float32, None, "delta", self.device)
        if delta.numel() != self.batch * self.n ** 3:
            raise ValueError("delta must hold batch * n^3 values")
        return self._rc(self.lib.recon_set_delta(self.handle, _ptr(delta)))

    def solve(self, start=START_PLAIN, net=None):
        if net is not None:
            _check_dev(net, torch.float32, None, "net", self.device)
            if net.numel() != CNN_PARAMS:
                raise ValueError(f"net must hold {CNN_PARAMS} parameters")
        return self._rc(self.lib.recon_solve(self.handle, int(start), _ptr(net)))

    def iterate(self, max_iter, tol):
        """Returns (code, passes per realisation, eps history [batch][<=max_iter]).  The code is
        RECON_OK, RECON_NOTCONVERGED, or RECON_RESTARTED when a rejected learned start restarted from
        the plain start (see restarts())."""
        iters = (ctypes.c_int32 * self.batch)()
        eps = (ctypes.c_double * (self.batch * max(max_iter, 1)))()
        rc = self._rc(self.lib.recon_iterate(self.handle, int(max_iter), float(tol), iters, eps),
                      allow=(RECON_OK, RECON_NOTCONVERGED, RECON_RESTARTED))
        hist = []
        for b in range(self.batch):
            row = [eps[b * max_iter + i] for i in range(max_iter)]
            hist.append([e for e in row if not math.isnan(e)])
        return rc, list(iters), hist

    def tile_counts(self):
        """Per realisation: (galaxy-grid tiles with data, random-grid tiles with data, tiles inside the mask,
        tiles), the z tiles of the last solve's transforms."""
        out = (ctypes.c_int64 * (4 * self.batch))()
        self._rc(self.lib.recon_tile_counts(self.handle, out))
        return [tuple(out[4 * b:4 * b + 4]) for b in range(self.batch)]

    def restarts(self):
        """Restarts from the plain start of each realisation since the last solve."""
        out = (ctypes.c_int32 * self.batch)()
        self._rc(self.lib.recon_start_restarts(self.handle, out))
        return list(out)

    def shift(self, which, pos, offsets=None, want_pos=False, out_disp=None, out_pos=None):
        if which not in (GAL, RAN):
            raise ValueError("which must be GAL or RAN")
        _check_dev(pos, torch.float32, (3,), "pos", self.device)
        self._check_offsets(offsets, pos.shape[0])
        disp = torch.empty_like(pos) if out_disp is None else out_disp
        out = (torch.empty_like(pos) if out_pos is None else out_pos) if want_pos else None
        _check_dev(disp, torch.float32, (3,), "out_disp", self.device)
        if out is not None:
            _check_dev(out, torch.float32, (3,), "out_pos", self.device)
        if disp.shape != pos.shape or (out is not None and out.shape != pos.shape):
            raise ValueError("output buffers must match pos")
        sel = which | (SHIFT_AS_PAINTED if self._as_painted(which, pos, offsets) else 0)
        self._rc(self.lib.recon_shift(self.handle, sel, _ptr(pos), pos.shape[0], _ptr(offsets), _ptr(disp),
                                      _ptr(out)))
        return (disp, out) if want_pos else disp

    def profile_start(self):
        return self._rc(self.lib.recon_profile_start(self.handle))

    def profile_stop(self):
        """Per-kernel {name: (launches, total_ms)} recorded since profile_start."""
        cap = 64
        counts = (ctypes.c_int32 * cap)()
        tot = (ctypes.c_double * cap)()
        k = self.lib.recon_profile_stop(self.handle, counts, tot, cap)
        if k < 0:
            self._rc(k)
        out = {}
        for i in range(min(k, cap)):
            if counts[i]:
                out[self.lib.recon_profile_kernel_name(i).decode()] = (int(counts[i]), float(tot[i]))
        return out

    def radial(self):
        """u = Psi . r_hat of the current displacement, [batch, n, n, n]."""
        out = torch.empty((self.batch, self.n, self.n, self.n), dtype=torch.float32, device=self.device)
        self._rc(self.lib.recon_get_radial(self.handle, _ptr(out)))
        return out

    def restrict(self, fine):
        """Full-weighting restriction [batch, n, n, n] -> [batch, n/2, n/2, n/2]."""
        _check_dev(fine, torch.float32, None, "fine", self.device)
        if fine.numel() != self.batch * self.n ** 3:
            raise ValueError("fine must hold batch * n^3 values")
        m = self.n // 2
        out = torch.empty((self.batch, m, m, m), dtype=torch.float32, device=self.device)
        self._rc(self.lib.recon_restrict(self.handle, _ptr(fine), _ptr(out)))
        return out

    def prolong(self, coarse):
        """Linear prolongation [batch, n/2, n/2, n/2] -> [batch, n, n, n]."""
        _check_dev(coarse, torch.float32, None, "coarse", self.device)
        if coarse.numel() != self.batch * (self.n // 2) ** 3:
            raise ValueError("coarse must hold batch * (n/2)^3 values")
        out = torch.empty((self.batch, self.n, self.n, self.n), dtype=torch.float32, device=self.device)
        self._rc(self.lib.recon_prolong(self.handle, _ptr(coarse), _ptr(out)))
        return out

    def cnn_forward(self, params, delta, u_p):
        """Learned radial correction Delta u on the network grid, [batch, m, m, m]."""
        for t, nm in ((params, "params"), (delta, "delta"), (u_p, "u_p")):
            _check_dev(t, torch.float32, None, nm, self.device)
        m = self.cnn_n
        if params.numel() != CNN_PARAMS or delta.numel() != self.batch * m ** 3 or u_p.numel() != delta.numel():
            raise ValueError("bad network input sizes")
        out = torch.empty((self.batch, m, m, m), dtype=torch.float32, device=self.device)
        self._rc(self.lib.recon_cnn_forward(self.handle, _ptr(params), _ptr(delta), _ptr(u_p), _ptr(out)))
        return out

    def cnn_train_step(self, params, m, v, step, lr, delta, u_p, target_du, grad_out=None):
        """One loss/gradient evaluation and (lr > 0) Adam update in place; returns the loss."""
        for t, nm in ((params, "params"), (delta, "delta"), (u_p, "u_p"), (target_du, "target_du")):
            _check_dev(t, torch.float32, None, nm, self.device)
        m3 = self.batch * self.cnn_n ** 3
        if params.numel() != CNN_PARAMS or any(t.numel() != m3 for t in (delta, u_p, target_du)):
            raise ValueError("bad network input sizes")
        vecs = ((m, "m"), (v, "v"), (grad_out, "grad_out")) if lr > 0 else ((grad_out, "grad_out"),)
        if lr > 0 and (m is None or v is None):
            raise ValueError("an Adam update needs the moment vectors m and v")
        for t, nm in vecs:
            if t is not None:
                _check_dev(t, torch.float32, None, nm, self.device)
                if t.numel() != CNN_PARAMS:
                    raise ValueError(f"{nm} must hold {CNN_PARAMS} values")
        loss = ctypes.c_double(0.0)
        self._rc(self.lib.recon_cnn_train_step(self.handle, _ptr(params), _ptr(m), _ptr(v), int(step), float(lr),
                                               _ptr(delta), _ptr(u_p), _ptr(target_du), ctypes.byref(loss),
                                               _ptr(grad_out)))
        return loss.value

    def psi(self):
        out = torch.empty((self.batch, 3, self.n, self.n, self.n), dtype=torch.float32, device=self.device)
        self._rc(self.lib.recon_get_psi(self.handle, _ptr(out)))
        return out

    def grid(self, which):
        out = torch.empty((self.batch, self.n, self.n, self.n), dtype=torch.int64, device=self.device)
        self._rc(self.lib.recon_get_grid(self.handle, which, _ptr(out)))
        return out

    def delta(self):
        out = torch.empty((self.batch, self.n, self.n, self.n), dtype=torch.float32, device=self.device)
        self._rc(self.lib.recon_get_delta(self.handle, _ptr(out)))
        return out


def plan_for(cat, **kw):
    """Plan matching a synthetic catalogue's geometry (binned deposit sized for its largest catalogue)."""
    if "max_objects" not in kw:
        kw["max_objects"] = max(cat.gal_pos.shape[0], 0 if cat.ran_pos is None else cat.ran_pos.shape[0])
    return Plan(cat.n, cat.box_len, cat.observer, cat.bias, cat.growth, cat.smooth_r, origin=cat.origin,
                mask_tau=cat.mask_tau, randoms=cat.ran_pos is not None, **kw)
