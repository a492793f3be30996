"""ctypes binding of libjt (include/jt.h): argument marshalling only.

Every step of the simulation runs in libjt's HIP kernels; this module turns
Python parameter objects and torch CUDA tensors into the C structs and device
pointers of the ABI, passes torch's current HIP stream, and raises `JtError`
for any non-OK status.  There is no fallback: if libjt.so has not been built the
first call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_uint64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjt.so")

JT_OK, JT_EINVAL, JT_ENOMEM, JT_EDEVICE, JT_EUNSUPPORTED, JT_EBUSY, JT_ECANCELLED = range(7)
STATUS_NAMES = {0: "JT_OK", 1: "JT_EINVAL", 2: "JT_ENOMEM", 3: "JT_EDEVICE", 4: "JT_EUNSUPPORTED",
                5: "JT_EBUSY", 6: "JT_ECANCELLED"}
JT_K_PREP, JT_K_RAY, JT_K_SB, JT_K_SIM, JT_K_CONV, JT_K_GRAD = range(6)
KERNEL_IDS = {"prep": JT_K_PREP, "ray": JT_K_RAY, "sb": JT_K_SB, "sim": JT_K_SIM, "conv": JT_K_CONV,
              "grad": JT_K_GRAD}


class JtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


# ---------------------------------------------------------------- C structs
class JtGrid(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("supersample", c_int),
                ("pixel_scale", c_double), ("x0", c_double), ("y0", c_double)]


class JtSie(ctypes.Structure):
    _fields_ = [("theta_E", c_double), ("q", c_double), ("phi", c_double), ("cx", c_double), ("cy", c_double)]


class JtShear(ctypes.Structure):
    _fields_ = [("gamma1", c_double), ("gamma2", c_double)]


class JtNfw(ctypes.Structure):
    _fields_ = [("n", c_int), ("x", c_void_p), ("y", c_void_p), ("Rs", c_void_p), ("alpha_Rs", c_void_p),
                ("r_trunc", c_void_p)]


class JtPointMasses(ctypes.Structure):
    _fields_ = [("n", c_int), ("x", POINTER(c_double)), ("y", POINTER(c_double)), ("theta_E", POINTER(c_double))]


class JtEpl(ctypes.Structure):
    _fields_ = [("theta_E", c_double), ("gamma", c_double), ("q", c_double), ("phi", c_double), ("cx", c_double),
                ("cy", c_double)]


def _epl(e):
    return JtEpl(e.theta_E, e.gamma, e.q, e.phi, e.cx, e.cy)


class JtLens(ctypes.Structure):
    _fields_ = [("has_sie", c_int), ("has_shear", c_int), ("sie", JtSie), ("shear", JtShear),
                ("nfw", JtNfw), ("subhalo_handle", c_uint64), ("pm", JtPointMasses),
                ("has_epl", c_int), ("epl", JtEpl)]


class JtSersic(ctypes.Structure):
    _fields_ = [("amp", c_double), ("R_sersic", c_double), ("n_sersic", c_double), ("q", c_double),
                ("phi", c_double), ("cx", c_double), ("cy", c_double)]


class JtGaussian(ctypes.Structure):
    _fields_ = [("amp", c_double), ("sigma", c_double), ("q", c_double), ("phi", c_double), ("cx", c_double),
                ("cy", c_double)]


class JtCoreSersic(ctypes.Structure):
    _fields_ = [("amp", c_double), ("R_sersic", c_double), ("R_b", c_double), ("n_sersic", c_double),
                ("gamma", c_double), ("alpha", c_double), ("q", c_double), ("phi", c_double), ("cx", c_double),
                ("cy", c_double)]


class JtShapelets(ctypes.Structure):
    _fields_ = [("n_max", c_int), ("beta", c_double), ("cx", c_double), ("cy", c_double),
                ("coeff", POINTER(c_double))]


class JtLight(ctypes.Structure):
    _fields_ = [("n", c_int), ("c", POINTER(JtSersic)), ("bn_exact", c_int), ("n_gauss", c_int),
                ("gauss", POINTER(JtGaussian)), ("n_core", c_int), ("core", POINTER(JtCoreSersic)),
                ("shapelets", POINTER(JtShapelets))]


class JtDraws(ctypes.Structure):
    _fields_ = [("B", c_int), ("sie", POINTER(JtSie)), ("shear", POINTER(JtShear)), ("n_sub", c_int),
                ("sub_x", c_void_p), ("sub_y", c_void_p), ("sub_Rs", c_void_p), ("sub_alpha_Rs", c_void_p),
                ("n_src", c_int), ("n_ll", c_int), ("src", POINTER(JtSersic)), ("ll", POINTER(JtSersic)),
                ("epl", POINTER(JtEpl)), ("sub_r_trunc", c_void_p)]


class JtFitProblem(ctypes.Structure):
    _fields_ = [("n_src", c_int), ("n_ll", c_int), ("lower", POINTER(c_double)), ("upper", POINTER(c_double)),
                ("n_sub", c_int), ("sub_x", c_void_p), ("sub_y", c_void_p), ("sub_Rs", c_void_p),
                ("sub_alpha_Rs", c_void_p), ("psf", c_void_p), ("k", c_int), ("data", c_void_p), ("inv_var", c_void_p)]


class JtPsoCfg(ctypes.Structure):
    _fields_ = [("n_particles", c_int), ("n_iterations", c_int), ("inertia", c_double), ("c_cognitive", c_double),
                ("c_social", c_double), ("seed", c_uint64)]


class JtLbfgsCfg(ctypes.Structure):
    _fields_ = [("starts", c_int), ("memory", c_int), ("max_iter", c_int), ("ftol", c_double), ("gtol", c_double)]


class JtServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_batch_images", c_int), ("max_batch_pairs", c_double),
                ("max_inflight_batches", c_int), ("n_streams", c_int)]


class JtRequest(ctypes.Structure):
    _fields_ = [("grid", JtGrid), ("has_sie", c_int), ("has_shear", c_int), ("sie", JtSie), ("shear", JtShear),
                ("subhalo_handle", c_uint64), ("src", JtLight), ("lens_light", JtLight), ("psf_handle", c_uint64),
                ("out", c_void_p), ("has_epl", c_int), ("epl", JtEpl)]


class JtServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_uint64), ("completed", c_uint64), ("cancelled", c_uint64), ("failed", c_uint64),
                ("batches", c_uint64), ("arena_bytes", c_uint64), ("arena_in_use", c_uint64),
                ("arena_peak", c_uint64), ("device_seconds", c_double), ("wait_seconds", c_double),
                ("run_seconds", c_double), ("max_wait_seconds", c_double)]


TICKET_QUEUED, TICKET_RUNNING, TICKET_DONE, TICKET_CANCELLED, TICKET_FAILED = range(5)


# ---------------------------------------------------------------- library
_LIB = None

_SIGS = {
    "jt_create": (c_int, [c_int, POINTER(c_void_p)]),
    "jt_destroy": (None, [c_void_p]),
    "jt_last_error": (c_char_p, []),
    "jt_version": (c_char_p, []),
    "jt_sync": (c_int, [c_void_p, c_void_p]),
    "jt_ray_shoot": (c_int, [c_void_p, c_int, c_void_p, c_void_p, POINTER(JtLens), c_void_p, c_void_p, c_void_p]),
    "jt_deflection": (c_int, [c_void_p, c_int, c_void_p, c_void_p, POINTER(JtLens), c_void_p, c_void_p, c_void_p]),
    "jt_source_sb": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(JtLight),
                             POINTER(JtLight), c_void_p, c_void_p]),
    "jt_convolve": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "jt_convolve_auto_method": (c_int, [c_int, c_int, c_int]),
    "jt_simulate_image": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtLens), POINTER(JtLight), POINTER(JtLight),
                                  c_void_p, c_int, c_void_p, c_void_p]),
    "jt_simulate_image_noalloc": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtLens), POINTER(JtLight),
                                          POINTER(JtLight), c_void_p, c_int, c_void_p, c_void_p]),
    "jt_calibrate_valu": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p]),
    "jt_upload_subhalos": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_uint64)]),
    "jt_linear_amplitudes": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtLens), POINTER(JtLight), POINTER(JtLight),
                                     c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "jt_pso": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtFitProblem), POINTER(JtPsoCfg), POINTER(c_double),
                       POINTER(c_double), POINTER(c_double), c_void_p]),
    "jt_pso_move": (c_int, [c_int, c_int, c_int, c_uint64, c_double, c_double, c_double, POINTER(c_double),
                            POINTER(c_double), POINTER(c_double), POINTER(c_double), POINTER(c_double),
                            POINTER(c_double)]),
    "jt_uniform": (c_double, [c_uint64, c_uint64]),
    "jt_lbfgs": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtFitProblem), POINTER(JtLbfgsCfg), POINTER(c_double),
                         POINTER(c_double), POINTER(c_double), POINTER(c_int), c_void_p]),
    "jt_upload_tnfw": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               POINTER(c_uint64)]),
    "jt_upload_psf": (c_int, [c_void_p, c_void_p, c_int, POINTER(c_uint64)]),
    "jt_psf_pointer": (c_int, [c_void_p, c_uint64, POINTER(c_void_p), POINTER(c_int)]),
    "jt_release": (c_int, [c_void_p, c_uint64]),
    "jt_profile_enable": (c_int, [c_void_p, c_int]),
    "jt_profile_read": (c_int, [c_void_p, c_int, POINTER(c_double), POINTER(c_int)]),
    "jt_sersic_bn": (c_double, [c_double, c_int]),
    "jt_simulate_batch": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtDraws), c_void_p, c_int, c_void_p, c_void_p]),
    "jt_chi2": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtDraws), c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                        c_void_p]),
    "jt_chi2_grad": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtDraws), c_void_p, c_int, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p, c_void_p]),
    "jt_chi2_grad_kept": (c_int, [c_void_p, POINTER(JtGrid), POINTER(JtDraws), c_void_p, c_int, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p]),
    "jt_server_create": (c_int, [c_void_p, POINTER(JtServerCfg), POINTER(c_void_p)]),
    "jt_server_create_simulated": (c_int, [POINTER(JtServerCfg), c_double, POINTER(c_void_p)]),
    "jt_server_simulate_failure": (c_int, [c_void_p, c_uint64]),
    "jt_server_submit": (c_int, [c_void_p, POINTER(JtRequest), POINTER(c_uint64)]),
    "jt_server_poll": (c_int, [c_void_p, c_uint64, POINTER(c_int)]),
    "jt_server_wait": (c_int, [c_void_p, c_uint64, c_double, POINTER(c_double)]),
    "jt_server_cancel": (c_int, [c_void_p, c_uint64]),
    "jt_server_get_stats": (c_int, [c_void_p, POINTER(JtServerStats)]),
    "jt_server_destroy": (None, [c_void_p]),
}


def load_library(path: str = LIB_PATH):
    """Load libjt.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libjt.so not found at {path}; build it with __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(status):
    if status != JT_OK:
        msg = load_library().jt_last_error()
        raise JtError(status, msg.decode() if msg else "")


def sersic_bn(n: float, exact: bool = False) -> float:
    """b_n as the library computes it on the host (FP64)."""
    return float(load_library().jt_sersic_bn(float(n), int(bool(exact))))


def convolve_auto_method(nx: int, ny: int, k: int) -> int:
    """The convolution path method 0 takes: 1 direct, 2 FFT, 0 none."""
    return int(load_library().jt_convolve_auto_method(int(nx), int(ny), int(k)))


def uniform(seed: int, i: int) -> float:
    """The library's counter-based uniform (SplitMix64 output i of `seed`)."""
    return float(load_library().jt_uniform(int(seed), int(i)))


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


def pso_move(t, seed, w, c1, c2, lower, upper, x, v, pbest, gbest):
    """The library's swarm update at step t on host arrays (x, v updated in place)."""
    N, P = x.shape
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (lower, upper, pbest, gbest)]
    if x.dtype != np.float64 or v.dtype != np.float64 or not x.flags.c_contiguous or not v.flags.c_contiguous:
        raise ValueError("x and v must be C-contiguous float64")
    _check(load_library().jt_pso_move(int(N), int(P), int(t), int(seed), float(w), float(c1), float(c2),
                                      _dptr(arrs[0]), _dptr(arrs[1]), _dptr(x), _dptr(v), _dptr(arrs[2]),
                                      _dptr(arrs[3])))


# ---------------------------------------------------------------- helpers
def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _dev_f32(a, device, keep):
    """Device float32 contiguous tensor view/copy of `a` (tensor or array)."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a
        if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
            t = t.to(device=device, dtype=torch.float32).contiguous()
    else:
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).to(device)
    keep.append(t)
    return t


def _require_out(t, shape, device):
    torch = _torch()
    if t is None:
        return torch.empty(shape, dtype=torch.float32, device=device)
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda" or tuple(t.shape) != tuple(shape):
        raise ValueError("output tensor must be a contiguous float32 CUDA tensor of shape %s" % (shape,))
    return t


class Context:
    """One libjt context on one HIP device."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self._lib = load_library()
        self.device = torch.device("cuda", device)
        self._ptr = c_void_p()
        _check(self._lib.jt_create(int(device), byref(self._ptr)))

    # lifetime
    def close(self):
        if self._ptr:
            self._lib.jt_destroy(self._ptr)
            self._ptr = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self, stream=None):
        _check(self._lib.jt_sync(self._ptr, _stream_handle(stream)))

    # ---- parameter marshalling
    def _lens(self, lens, keep):
        L = JtLens()
        sie = getattr(lens, "sie", None)
        if sie is not None:
            L.has_sie = 1
            L.sie = JtSie(sie.theta_E, sie.q, sie.phi, sie.cx, sie.cy)
        sh = getattr(lens, "shear", None)
        if sh is not None:
            L.has_shear = 1
            L.shear = JtShear(sh.gamma1, sh.gamma2)
        epl = getattr(lens, "epl", None)
        if epl is not None:
            L.has_epl = 1
            L.epl = _epl(epl)
        handle = getattr(lens, "subhalo_handle", 0) or 0
        nfw = getattr(lens, "nfw", None)
        if handle:
            L.subhalo_handle = int(handle)
        elif nfw is not None and len(nfw.x) > 0:
            rt = getattr(nfw, "r_trunc", None)
            fields = (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs) + ((rt,) if rt is not None else ())
            arrs = [_dev_f32(a, self.device, keep) for a in fields]
            L.nfw = JtNfw(int(arrs[0].numel()), *[c_void_p(a.data_ptr()) for a in arrs])
        pm = getattr(lens, "point_masses", None)
        if pm is not None and np.size(pm.x) > 0:
            cols = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1)) for v in (pm.x, pm.y, pm.theta_E)]
            keep.extend(cols)
            ptrs = [c.ctypes.data_as(POINTER(c_double)) for c in cols]
            L.pm = JtPointMasses(int(cols[0].size), *ptrs)
        return L

    @staticmethod
    def _light(comps, bn_exact, keep):
        """A jt_light from a list of components, sorted by profile: Sersic
        (amp, R_sersic, n_sersic, ...), Gaussian (sigma), core-Sersic (R_b)
        and at most one shapelet set (coeff)."""
        comps = list(comps or [])
        sh = [c for c in comps if hasattr(c, "coeff")]
        ga = [c for c in comps if hasattr(c, "sigma")]
        co = [c for c in comps if hasattr(c, "R_b")]
        se = [c for c in comps if not (hasattr(c, "coeff") or hasattr(c, "sigma") or hasattr(c, "R_b"))]
        if len(sh) > 1:
            raise ValueError("at most one shapelet set per light list")
        arr = (JtSersic * max(1, len(se)))()
        for i, c in enumerate(se):
            arr[i] = JtSersic(c.amp, c.R_sersic, c.n_sersic, c.q, c.phi, c.cx, c.cy)
        garr = (JtGaussian * max(1, len(ga)))()
        for i, c in enumerate(ga):
            garr[i] = JtGaussian(c.amp, c.sigma, c.q, c.phi, c.cx, c.cy)
        carr = (JtCoreSersic * max(1, len(co)))()
        for i, c in enumerate(co):
            carr[i] = JtCoreSersic(c.amp, c.R_sersic, c.R_b, c.n_sersic, c.gamma, c.alpha, c.q, c.phi, c.cx, c.cy)
        keep.extend([arr, garr, carr])
        L = JtLight(len(se), ctypes.cast(arr, POINTER(JtSersic)), int(bool(bn_exact)), len(ga),
                    ctypes.cast(garr, POINTER(JtGaussian)), len(co), ctypes.cast(carr, POINTER(JtCoreSersic)), None)
        if sh:
            s0 = sh[0]
            coeff = np.ascontiguousarray(np.asarray(s0.coeff, dtype=np.float64))
            if coeff.size != (s0.n_max + 1) * (s0.n_max + 2) // 2:
                raise ValueError("shapelet coefficients must number (n_max + 1)(n_max + 2)/2")
            S = JtShapelets(int(s0.n_max), float(s0.beta), float(s0.cx), float(s0.cy),
                            coeff.ctypes.data_as(POINTER(c_double)))
            keep.extend([coeff, S])
            L.shapelets = ctypes.pointer(S)
        return L

    # ---- step 1
    def _ray(self, fn, x, y, lens, out, stream):
        keep = []
        xt = _dev_f32(x, self.device, keep)
        yt = _dev_f32(y, self.device, keep)
        n = xt.numel()
        ox = _require_out(out[0] if out else None, xt.shape, self.device)
        oy = _require_out(out[1] if out else None, yt.shape, self.device)
        L = self._lens(lens, keep)
        _check(fn(self._ptr, n, c_void_p(xt.data_ptr()), c_void_p(yt.data_ptr()), byref(L),
                  c_void_p(ox.data_ptr()), c_void_p(oy.data_ptr()), _stream_handle(stream)))
        self._retain(keep, stream)
        return ox, oy

    def ray_shoot(self, x, y, lens, out=None, stream=None):
        """beta = theta - alpha(theta) at the points (x, y)."""
        return self._ray(self._lib.jt_ray_shoot, x, y, lens, out, stream)

    def deflection(self, x, y, lens, out=None, stream=None):
        """alpha(theta) at the points (x, y)."""
        return self._ray(self._lib.jt_deflection, x, y, lens, out, stream)

    # ---- step 2
    def source_sb(self, x, y, bx, by, source, lens_light=(), bn_exact=False, out=None, stream=None):
        keep = []
        bxt = _dev_f32(bx, self.device, keep)
        byt = _dev_f32(by, self.device, keep)
        xt = _dev_f32(x, self.device, keep) if x is not None else bxt
        yt = _dev_f32(y, self.device, keep) if y is not None else byt
        sb = _require_out(out, bxt.shape, self.device)
        S = self._light(source, bn_exact, keep)
        LL = self._light(lens_light, bn_exact, keep)
        _check(self._lib.jt_source_sb(self._ptr, bxt.numel(), c_void_p(xt.data_ptr()), c_void_p(yt.data_ptr()),
                                      c_void_p(bxt.data_ptr()), c_void_p(byt.data_ptr()), byref(S), byref(LL),
                                      c_void_p(sb.data_ptr()), _stream_handle(stream)))
        self._retain(keep, stream)
        return sb

    # ---- step 3
    def convolve(self, img, psf, method=0, out=None, stream=None):
        keep = []
        it = _dev_f32(img, self.device, keep)
        pt = _dev_f32(psf, self.device, keep)
        if it.dim() != 2 or pt.dim() != 2 or pt.shape[0] != pt.shape[1]:
            raise ValueError("convolve: image must be 2-D and the PSF square")
        ny, nx = it.shape
        o = _require_out(out, (ny, nx), self.device)
        _check(self._lib.jt_convolve(self._ptr, c_void_p(it.data_ptr()), int(nx), int(ny), c_void_p(pt.data_ptr()),
                                     int(pt.shape[0]), int(method), c_void_p(o.data_ptr()), _stream_handle(stream)))
        self._retain(keep, stream)
        return o

    # ---- fused
    def simulate_image(self, grid, lens, source, lens_light=(), psf=None, bn_exact=False, out=None, stream=None,
                       noalloc=False):
        """The fused simulation (jt_simulate_image).  noalloc=True calls
        jt_simulate_image_noalloc, whose intermediates live in the library's
        static per-device scratch (direct convolution only)."""
        keep = []
        G = JtGrid(int(grid.nx), int(grid.ny), int(grid.supersample), float(grid.pixel_scale),
                   float(grid.x0), float(grid.y0))
        L = self._lens(lens, keep)
        S = self._light(source, bn_exact, keep)
        LL = self._light(lens_light, bn_exact, keep)
        o = _require_out(out, (int(grid.ny), int(grid.nx)), self.device)
        if psf is None:
            pp, k = c_void_p(), 0
        else:
            pt = _dev_f32(psf, self.device, keep)
            pp, k = c_void_p(pt.data_ptr()), int(pt.shape[0])
        fn = self._lib.jt_simulate_image_noalloc if noalloc else self._lib.jt_simulate_image
        _check(fn(self._ptr, byref(G), byref(L), byref(S), byref(LL), pp, k, c_void_p(o.data_ptr()),
                  _stream_handle(stream)))
        self._retain(keep, stream)
        return o

    def simulate_scene(self, scene, psf=True, **kw):
        """simulate_image for a workloads.Scene-like object."""
        return self.simulate_image(scene.grid, scene.lens, scene.source, scene.lens_light,
                                   scene.psf if psf else None, getattr(scene, "bn_exact", False), **kw)

    # ---- linear amplitude solver
    def linear_amplitudes(self, grid, lens, source, lens_light, data, inv_var, psf=None, bn_exact=False,
                          model=True, stream=None):
        """Weighted least-squares amplitudes of the light components (sources,
        then lens light; their amp fields are ignored) for the image `data`
        with weights `inv_var`.  Returns (amps float64 [n], model float32
        [ny, nx] or None, logL float64 [1]) as device tensors."""
        torch = _torch()
        keep = []
        G = JtGrid(int(grid.nx), int(grid.ny), int(grid.supersample), float(grid.pixel_scale),
                   float(grid.x0), float(grid.y0))
        L = self._lens(lens, keep)
        S = self._light(source, bn_exact, keep)
        LL = self._light(lens_light, bn_exact, keep)
        shape = (int(grid.ny), int(grid.nx))
        dt = _dev_f32(data, self.device, keep)
        wt = _dev_f32(inv_var, self.device, keep)
        if tuple(dt.shape) != shape or tuple(wt.shape) != shape:
            raise ValueError("data and inv_var must be [ny, nx]")
        if psf is None:
            pp, k = c_void_p(), 0
        else:
            pt = _dev_f32(psf, self.device, keep)
            pp, k = c_void_p(pt.data_ptr()), int(pt.shape[0])
        n = len(source) + len(lens_light)
        amps = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        mo = torch.empty(shape, dtype=torch.float32, device=self.device) if model else None
        logL = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(self._lib.jt_linear_amplitudes(self._ptr, byref(G), byref(L), byref(S), byref(LL), pp, k,
                                              c_void_p(dt.data_ptr()), c_void_p(wt.data_ptr()),
                                              c_void_p(amps.data_ptr()),
                                              c_void_p(mo.data_ptr() if mo is not None else None),
                                              c_void_p(logL.data_ptr()), _stream_handle(stream)))
        self._retain(keep, stream)
        return amps[:n], mo, logL

    # ---- fitting loops
    def _fit_problem(self, n_src, n_ll, lower, upper, data, inv_var, psf, nfw, keep):
        lo = np.ascontiguousarray(np.asarray(lower, dtype=np.float64))
        hi = np.ascontiguousarray(np.asarray(upper, dtype=np.float64))
        keep.extend([lo, hi])
        Pr = JtFitProblem()
        Pr.n_src, Pr.n_ll = int(n_src), int(n_ll)
        Pr.lower, Pr.upper = _dptr(lo), _dptr(hi)
        if nfw is not None and len(nfw.x) > 0:
            arrs = [_dev_f32(a, self.device, keep) for a in (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs)]
            Pr.n_sub = int(arrs[0].numel())
            Pr.sub_x, Pr.sub_y, Pr.sub_Rs, Pr.sub_alpha_Rs = [c_void_p(a.data_ptr()) for a in arrs]
        if psf is not None:
            pt = _dev_f32(psf, self.device, keep)
            Pr.psf, Pr.k = c_void_p(pt.data_ptr()), int(pt.shape[0])
        Pr.data = c_void_p(_dev_f32(data, self.device, keep).data_ptr())
        Pr.inv_var = c_void_p(_dev_f32(inv_var, self.device, keep).data_ptr())
        return Pr, lo.size

    def pso(self, grid, n_src, n_ll, lower, upper, data, inv_var, psf=None, nfw=None, n_particles=64,
            n_iterations=100, inertia=0.7298, c_cognitive=1.49618, c_social=1.49618, seed=0, stream=None):
        """Particle swarm maximising log L over the box; returns (best [P],
        best log L, history [n_iterations]) on the host."""
        keep = []
        G = JtGrid(int(grid.nx), int(grid.ny), int(grid.supersample), float(grid.pixel_scale),
                   float(grid.x0), float(grid.y0))
        Pr, P = self._fit_problem(n_src, n_ll, lower, upper, data, inv_var, psf, nfw, keep)
        cfg = JtPsoCfg(int(n_particles), int(n_iterations), float(inertia), float(c_cognitive), float(c_social),
                       int(seed))
        best = np.empty(P)
        hist = np.empty(max(int(n_iterations), 1))
        bl = c_double()
        _check(self._lib.jt_pso(self._ptr, byref(G), byref(Pr), byref(cfg), _dptr(best), byref(bl), _dptr(hist),
                                _stream_handle(stream)))
        return best, bl.value, hist[:int(n_iterations)]

    def lbfgs(self, grid, n_src, n_ll, lower, upper, data, inv_var, x0, psf=None, nfw=None, memory=10,
              max_iter=200, ftol=1e-12, gtol=1e-10, stream=None):
        """L-BFGS chains minimising -log L from the rows of x0 [starts, P];
        returns (x [starts, P], log L [starts], iterations [starts])."""
        keep = []
        G = JtGrid(int(grid.nx), int(grid.ny), int(grid.supersample), float(grid.pixel_scale),
                   float(grid.x0), float(grid.y0))
        Pr, P = self._fit_problem(n_src, n_ll, lower, upper, data, inv_var, psf, nfw, keep)
        x0 = np.ascontiguousarray(np.atleast_2d(np.asarray(x0, dtype=np.float64)))
        if x0.shape[1] != P:
            raise ValueError(f"x0 rows must hold {P} values")
        C = x0.shape[0]
        cfg = JtLbfgsCfg(C, int(memory), int(max_iter), float(ftol), float(gtol))
        x = np.empty_like(x0)
        ll = np.empty(C)
        its = np.empty(C, dtype=np.int32)
        _check(self._lib.jt_lbfgs(self._ptr, byref(G), byref(Pr), byref(cfg), _dptr(x0), _dptr(x), _dptr(ll),
                                  its.ctypes.data_as(POINTER(c_int)), _stream_handle(stream)))
        return x, ll, its

    # ---- batches of parameter draws
    def _draws(self, batch, keep):
        """JtDraws from a DrawBatch (macro rows on the host, subhalo SoA on the
        device).  Macro row: SIE (5) or, with batch.main == "epl", EPL (6:
        theta_E, gamma, q, phi, cx, cy), then shear (2), then 7 per Sersic."""
        mac = np.ascontiguousarray(np.asarray(batch.macro, dtype=np.float64))
        B, P = mac.shape
        ns, nl = int(batch.n_src), int(batch.n_ll)
        epl = getattr(batch, "main", "sie") == "epl"
        m = 6 if epl else 5
        if P != m + 2 + 7 * (ns + nl):
            raise ValueError(f"macro rows must hold {m + 2} + 7 (n_src + n_ll) values")
        o = m + 2
        main = ((JtEpl * B)(*[JtEpl(*row[:6]) for row in mac]) if epl
                else (JtSie * B)(*[JtSie(*row[:5]) for row in mac]))
        sh = (JtShear * B)(*[JtShear(*row[m:m + 2]) for row in mac])
        src = (JtSersic * max(1, B * ns))(*[JtSersic(*row[o + 7 * k:o + 7 + 7 * k]) for row in mac
                                            for k in range(ns)])
        ll = (JtSersic * max(1, B * nl))(*[JtSersic(*row[o + 7 * (ns + k):o + 7 + 7 * (ns + k)])
                                           for row in mac for k in range(nl)])
        keep.extend([main, sh, src, ll])
        D = JtDraws()
        D.B = B
        if epl:
            D.epl = ctypes.cast(main, POINTER(JtEpl))
        else:
            D.sie = ctypes.cast(main, POINTER(JtSie))
        D.shear = ctypes.cast(sh, POINTER(JtShear))
        D.n_src, D.n_ll = ns, nl
        D.src = ctypes.cast(src, POINTER(JtSersic))
        D.ll = ctypes.cast(ll, POINTER(JtSersic)) if nl else None
        n = 0 if batch.sub_x is None else int(batch.sub_x.shape[-1])
        D.n_sub = n
        if n:
            arrs = [_dev_f32(a, self.device, keep) for a in (batch.sub_x, batch.sub_y, batch.sub_Rs, batch.sub_alpha_Rs)]
            for a in arrs:
                if tuple(a.shape) != (B, n):
                    raise ValueError("subhalo arrays must be [B, n_sub]")
            D.sub_x, D.sub_y, D.sub_Rs, D.sub_alpha_Rs = [c_void_p(a.data_ptr()) for a in arrs]
            rt = getattr(batch, "sub_r_trunc", None)
            if rt is not None:
                t = _dev_f32(rt, self.device, keep)
                if tuple(t.shape) != (B, n):
                    raise ValueError("sub_r_trunc must be [B, n_sub]")
                D.sub_r_trunc = c_void_p(t.data_ptr())
        return D, B, n, P

    @staticmethod
    def _grid(grid):
        return JtGrid(int(grid.nx), int(grid.ny), int(grid.supersample), float(grid.pixel_scale),
                      float(grid.x0), float(grid.y0))

    def _psf(self, psf, keep):
        if psf is None:
            return c_void_p(), 0
        pt = _dev_f32(psf, self.device, keep)
        return c_void_p(pt.data_ptr()), int(pt.shape[0])

    def simulate_batch(self, grid, batch, psf=None, out=None, stream=None):
        """Forward images of every draw: [B, ny, nx]."""
        keep = []
        D, B, _, _ = self._draws(batch, keep)
        G = self._grid(grid)
        o = _require_out(out, (B, int(grid.ny), int(grid.nx)), self.device)
        pp, k = self._psf(psf, keep)
        _check(self._lib.jt_simulate_batch(self._ptr, byref(G), byref(D), pp, k, c_void_p(o.data_ptr()),
                                           _stream_handle(stream)))
        self._retain(keep, stream)
        return o

    def chi2(self, grid, batch, data, inv_var, psf=None, stream=None):
        """log L of every draw (float64 [B])."""
        torch = _torch()
        keep = []
        D, B, _, _ = self._draws(batch, keep)
        G = self._grid(grid)
        pp, k = self._psf(psf, keep)
        dt = _dev_f32(data, self.device, keep)
        wt = _dev_f32(inv_var, self.device, keep)
        logL = torch.empty(B, dtype=torch.float64, device=self.device)
        _check(self._lib.jt_chi2(self._ptr, byref(G), byref(D), pp, k, c_void_p(dt.data_ptr()),
                                 c_void_p(wt.data_ptr()), c_void_p(logL.data_ptr()), _stream_handle(stream)))
        self._retain(keep, stream)
        return logL

    def chi2_grad(self, grid, batch, data, inv_var, psf=None, stream=None, keep_positions=False):
        """(log L [B] float64, d log L / d macro [B, P], d log L / d (x, y, alpha_Rs) [B, n, 3]).

        The backward pass recomputes the traced positions; with
        `keep_positions` the forward keeps them (8 bytes per sub-pixel per
        draw) and the backward reads them back, with identical results."""
        torch = _torch()
        keep = []
        D, B, n, P = self._draws(batch, keep)
        G = self._grid(grid)
        pp, k = self._psf(psf, keep)
        dt = _dev_f32(data, self.device, keep)
        wt = _dev_f32(inv_var, self.device, keep)
        logL = torch.empty(B, dtype=torch.float64, device=self.device)
        gm = torch.empty((B, P), dtype=torch.float32, device=self.device)
        gs = torch.empty((B, n, 3), dtype=torch.float32, device=self.device)
        fn = self._lib.jt_chi2_grad_kept if keep_positions else self._lib.jt_chi2_grad
        _check(fn(self._ptr, byref(G), byref(D), pp, k, c_void_p(dt.data_ptr()), c_void_p(wt.data_ptr()),
                  c_void_p(logL.data_ptr()), c_void_p(gm.data_ptr()), c_void_p(gs.data_ptr() if n else None),
                  _stream_handle(stream)))
        self._retain(keep, stream)
        return logL, gm, gs

    # ---- resident tables
    def upload_subhalos(self, nfw) -> int:
        """Resident table of NFW subhalos, or of truncated ones when
        `nfw.r_trunc` is set."""
        rt = getattr(nfw, "r_trunc", None)
        fields = (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs) + ((rt,) if rt is not None else ())
        cols = [np.ascontiguousarray(np.asarray(v, dtype=np.float32)) for v in fields]
        h = c_uint64()
        fn = self._lib.jt_upload_tnfw if rt is not None else self._lib.jt_upload_subhalos
        _check(fn(self._ptr, int(cols[0].size), *[c_void_p(c.ctypes.data) for c in cols], byref(h)))
        return int(h.value)

    def upload_psf(self, psf) -> int:
        p = np.ascontiguousarray(np.asarray(psf, dtype=np.float32))
        h = c_uint64()
        _check(self._lib.jt_upload_psf(self._ptr, c_void_p(p.ctypes.data), int(p.shape[0]), byref(h)))
        return int(h.value)

    def psf_pointer(self, handle: int):
        p, k = c_void_p(), c_int()
        _check(self._lib.jt_psf_pointer(self._ptr, c_uint64(handle), byref(p), byref(k)))
        return p.value, k.value

    def release(self, handle: int):
        _check(self._lib.jt_release(self._ptr, c_uint64(handle)))

    # ---- timing
    def profile_enable(self, on=True):
        _check(self._lib.jt_profile_enable(self._ptr, int(bool(on))))

    def calibrate_valu(self, kind: int, blocks: int, iters: int, reps: int = 3, stream=None):
        """Runs the FP32 issue-rate calibration kernel `kind` (jt_calibrate_valu)
        reps times; returns the fastest launch in milliseconds (HIP events on
        the launch stream)."""
        torch = _torch()
        out = torch.empty(int(blocks) * 256, dtype=torch.float32, device=self.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        best = float("inf")
        for _ in range(int(reps) + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            _check(self._lib.jt_calibrate_valu(int(kind), int(blocks), int(iters), c_void_p(out.data_ptr()),
                                               c_void_p(s.cuda_stream)))
            b.record(s)
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        if not torch.isfinite(out).all():
            raise RuntimeError("calibration chains did not stay finite")
        return best

    def profile_read(self, kernel: str):
        ms, n = c_double(), c_int()
        _check(self._lib.jt_profile_read(self._ptr, KERNEL_IDS[kernel], byref(ms), byref(n)))
        return ms.value, n.value

    # ---- internals
    def _retain(self, keep, stream):
        """Device copies made for a call must outlive the kernels that read
        them: mark them as used on the launch stream."""
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        for t in keep:
            if isinstance(t, torch.Tensor) and t.device.type == "cuda":
                t.record_stream(s)


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching server (jt_server_*).  `ctx=None` builds the
    simulated-device server used to test the scheduler without a GPU; its
    requests carry the subhalo count and PSF side in place of handles."""

    def __init__(self, ctx=None, hbm_budget_bytes=1 << 30, max_batch_images=64, max_batch_pairs=2e9,
                 max_inflight_batches=4, n_streams=4, simulated_pairs_per_s=None):
        self._lib = load_library()
        self.ctx = ctx
        cfg = JtServerCfg(int(hbm_budget_bytes), int(max_batch_images), float(max_batch_pairs),
                          int(max_inflight_batches), int(n_streams))
        self._ptr = c_void_p()
        if ctx is None:
            _check(self._lib.jt_server_create_simulated(byref(cfg), float(simulated_pairs_per_s or 1e12),
                                                        byref(self._ptr)))
        else:
            _check(self._lib.jt_server_create(ctx._ptr, byref(cfg), byref(self._ptr)))

    def close(self):
        if self._ptr:
            self._lib.jt_server_destroy(self._ptr)
            self._ptr = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, grid, lens, source, lens_light=(), out=None, subhalo_handle=0, psf_handle=0, bn_exact=False):
        """Queue one image; returns its ticket.  `out` is a device float32
        [ny, nx] tensor (any non-null address for the simulated server)."""
        keep = []
        R = JtRequest()
        R.grid = JtGrid(int(grid.nx), int(grid.ny), int(grid.supersample), float(grid.pixel_scale),
                        float(grid.x0), float(grid.y0))
        sie = getattr(lens, "sie", None)
        if sie is not None:
            R.has_sie = 1
            R.sie = JtSie(sie.theta_E, sie.q, sie.phi, sie.cx, sie.cy)
        sh = getattr(lens, "shear", None)
        if sh is not None:
            R.has_shear = 1
            R.shear = JtShear(sh.gamma1, sh.gamma2)
        epl = getattr(lens, "epl", None)
        if epl is not None:
            R.has_epl = 1
            R.epl = _epl(epl)
        R.subhalo_handle = int(subhalo_handle)
        R.psf_handle = int(psf_handle)
        R.src = Context._light(source, bn_exact, keep)
        R.lens_light = Context._light(lens_light, bn_exact, keep)
        if out is None:
            R.out = c_void_p(1)
        elif isinstance(out, int):
            R.out = c_void_p(out)
        else:
            R.out = c_void_p(out.data_ptr())
        t = c_uint64()
        _check(self._lib.jt_server_submit(self._ptr, byref(R), byref(t)))
        return int(t.value)

    def poll(self, ticket):
        st = c_int()
        _check(self._lib.jt_server_poll(self._ptr, c_uint64(ticket), byref(st)))
        return st.value

    def wait(self, ticket, timeout=-1.0):
        """Seconds from submission to completion; raises JtError when the
        ticket was cancelled, failed or is still pending at the timeout."""
        lat = c_double()
        _check(self._lib.jt_server_wait(self._ptr, c_uint64(ticket), float(timeout), byref(lat)))
        return lat.value

    def cancel(self, ticket):
        _check(self._lib.jt_server_cancel(self._ptr, c_uint64(ticket)))

    def simulate_failure(self, batch):
        """Simulated server: launch number `batch` (1-based) fails on completion."""
        _check(self._lib.jt_server_simulate_failure(self._ptr, c_uint64(int(batch))))

    def stats(self):
        s = JtServerStats()
        _check(self._lib.jt_server_get_stats(self._ptr, byref(s)))
        return {f: getattr(s, f) for f, _ in JtServerStats._fields_}
