"""Thin Python binding of the C ABI (argument marshalling only).

Every method has the name of the C call it wraps.  Arrays are torch tensors on
the GPU (float32, contiguous); torch supplies device memory and the current
stream, and nothing here computes on the data.
"""

import ctypes as C

from . import _lib
from ._lib import (tomo_rect, roi_params, tomo_launch, ROI_TV_NONNEG_CP, ROI_NONNEG_SIRT,
                   ROI_LOCAL_SIRT, ROI_LOCAL_FISTA_TV, ROI_LOCAL_FISTA_HAAR, ROI_FLAG_BOX)


class TomoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _rect(r):
    if isinstance(r, tomo_rect):
        return r
    return tomo_rect(*[int(v) for v in r])


def _ptr(t, shape=None, name="array", host=False):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.device.type != ("cpu" if host else "cuda"):
        raise ValueError(f"{name} must be on the {'host' if host else 'GPU'}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_params(roi, margin, method="cp", lam=0.0, iters=100, sigma=0.0, tau=0.0, flags=0,
                box=None, inner_iters=0):
    """roi_params; method "cp", "sirt", "local", "fista" or "haar" (or the enum value);
    box=(lo, hi) sets ROI_FLAG_BOX with those bounds; inner_iters: FGP iterations of
    "fista", Haar levels of "haar" (0: the library's default)."""
    m = {"cp": ROI_TV_NONNEG_CP, "sirt": ROI_NONNEG_SIRT, "local": ROI_LOCAL_SIRT,
         "fista": ROI_LOCAL_FISTA_TV, "haar": ROI_LOCAL_FISTA_HAAR}.get(method, method)
    lo, hi = 0.0, float("inf")
    if box is not None:
        lo, hi = float(box[0]), float(box[1])
        flags = int(flags) | ROI_FLAG_BOX
    return roi_params(_rect(roi), int(margin), int(m), float(lam), int(iters), float(sigma),
                      float(tau), int(flags), lo, hi, int(inner_iters))


class Context:
    """A library context on one GPU (device >= 0) or a host-only planning
    context (device = -1).  The workspace (a uint8 tensor) is the only device
    memory the library uses, and its size is the HBM budget of serving."""

    def __init__(self, device=0, workspace_bytes=1 << 30, workspace=None):
        self.lib = _lib.load()
        self._ws = None
        ptr, size = None, 0
        if device >= 0:
            import torch
            if workspace is None:
                workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8,
                                        device=f"cuda:{device}")
            self._ws = workspace
            ptr, size = C.c_void_p(workspace.data_ptr()), workspace.numel()
        h = C.c_void_p()
        st = self.lib.tomo_create(int(device), ptr, C.c_size_t(size), C.byref(h))
        if st != 0:
            raise TomoError(st, "tomo_create failed")
        self.h = h
        self.geoms = {}
        self.fake = False   # serving through the host test executor (host memory)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tomo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise TomoError(st, self.lib.tomo_last_error(self.h).decode())
        return st

    # -- geometry -------------------------------------------------------
    def tomo_set_geometry(self, n, n_angles, n_det, angles=None, det_spacing=1.0,
                          det_offset=0.0):
        gid = C.c_int32()
        arr = None
        if angles is not None:
            arr = (C.c_double * len(angles))(*[float(a) for a in angles])
        self._check(self.lib.tomo_set_geometry(self.h, n, n_angles, n_det, arr,
                                               float(det_spacing), float(det_offset),
                                               C.byref(gid)))
        self.geoms[gid.value] = (n, n_angles, n_det)
        return gid.value

    def tomo_roi_band(self, geom, region):
        na = self.geoms[geom][1]
        i0 = (C.c_int32 * na)()
        w = (C.c_int32 * na)()
        self._check(self.lib.tomo_roi_band(self.h, geom, _rect(region), i0, w))
        return list(i0), list(w)

    def tomo_roi_ext(self, geom, roi, margin):
        e = tomo_rect()
        self._check(self.lib.tomo_roi_ext(self.h, geom, _rect(roi), int(margin), C.byref(e)))
        return (e.row0, e.col0, e.rows, e.cols)

    # -- operators ------------------------------------------------------
    def tomo_fp(self, geom, region, img, sino, accumulate=False, stream=None):
        n, na, nd = self.geoms[geom]
        r = _rect(region)
        self._check(self.lib.tomo_fp(self.h, geom, r, _ptr(img, (r.rows, r.cols), "img"),
                                     _ptr(sino, (na, nd), "sino"), int(accumulate),
                                     _stream(stream)))

    def tomo_bp(self, geom, region, sino, img, accumulate=False, stream=None):
        n, na, nd = self.geoms[geom]
        r = _rect(region)
        self._check(self.lib.tomo_bp(self.h, geom, r, _ptr(sino, (na, nd), "sino"),
                                     _ptr(img, (r.rows, r.cols), "img"), int(accumulate),
                                     _stream(stream)))

    def tomo_fbp_ramlak(self, geom, sino, img, stream=None):
        n, na, nd = self.geoms[geom]
        self._check(self.lib.tomo_fbp_ramlak(self.h, geom, _ptr(sino, (na, nd), "sino"),
                                             _ptr(img, (n, n), "img"), _stream(stream)))

    def tomo_fbp_ramlak_noalloc(self, geom, sino, img, stream=None):
        n, na, nd = self.geoms[geom]
        self._check(self.lib.tomo_fbp_ramlak_noalloc(
            self.h, geom, _ptr(sino, (na, nd), "sino"), _ptr(img, (n, n), "img"),
            _stream(stream)))

    def tomo_exterior_subtract(self, geom, ext_roi, sino, x_ext, sino_local, stream=None):
        n, na, nd = self.geoms[geom]
        self._check(self.lib.tomo_exterior_subtract(
            self.h, geom, _rect(ext_roi), _ptr(sino, (na, nd), "sino"),
            _ptr(x_ext, (n, n), "x_ext"), _ptr(sino_local, (na, nd), "sino_local"),
            _stream(stream)))

    # -- solves ---------------------------------------------------------
    def roi_solve(self, geom, sino, params, out, x_ext=None, stream=None):
        n, na, nd = self.geoms[geom]
        p = params
        self._check(self.lib.roi_solve(self.h, geom, _ptr(sino, (na, nd), "sino"),
                                       _ptr(x_ext, (n, n), "x_ext"), C.byref(p),
                                       _ptr(out, (p.roi.rows, p.roi.cols), "out"),
                                       _stream(stream)))

    def roi_state_bytes(self, geom, params):
        b = C.c_size_t()
        self._check(self.lib.roi_state_bytes(self.h, geom, C.byref(params), C.byref(b)))
        return b.value

    def roi_solve_resume(self, geom, sino, params, done, state, out, x_ext=None, stream=None):
        """state: float32 GPU tensor of roi_state_bytes / 4 entries (caller-owned)."""
        n, na, nd = self.geoms[geom]
        p = params
        nbytes = self.roi_state_bytes(geom, p)
        self._check(self.lib.roi_solve_resume(self.h, geom, _ptr(sino, (na, nd), "sino"),
                                              _ptr(x_ext, (n, n), "x_ext"), C.byref(p),
                                              int(done), _ptr(state, (nbytes // 4,), "state"),
                                              _ptr(out, (p.roi.rows, p.roi.cols), "out"),
                                              _stream(stream)))

    def roi_solve_batch(self, geom, sino, params, outs, x_ext=None, stream=None):
        n, na, nd = self.geoms[geom]
        cnt = len(params)
        parr = (roi_params * cnt)(*params)
        oarr = (C.c_void_p * cnt)(*[_ptr(o, (p.roi.rows, p.roi.cols), "out").value
                                    for o, p in zip(outs, params)])
        self._check(self.lib.roi_solve_batch(self.h, geom, _ptr(sino, (na, nd), "sino"),
                                             _ptr(x_ext, (n, n), "x_ext"), cnt, parr, oarr,
                                             _stream(stream)))

    def roi_solve_stitched(self, geom, sino, params, img, x_ext=None, stream=None):
        """Batched solve with every ROI's crop written into img (a contiguous float32
        [n][ld] tensor, ld >= n) at the ROI's position."""
        n, na, nd = self.geoms[geom]
        cnt = len(params)
        parr = (roi_params * cnt)(*params)
        ptr = _ptr(img, None, "img")
        if img.dim() != 2 or img.shape[0] != n or img.shape[1] < n:
            raise ValueError(f"img has shape {tuple(img.shape)}, expected ({n}, >= {n})")
        self._check(self.lib.roi_solve_stitched(
            self.h, geom, _ptr(sino, (na, nd), "sino"), _ptr(x_ext, (n, n), "x_ext"), cnt, parr,
            ptr, int(img.shape[1]), _stream(stream)))

    # -- the paper's local method (Alg. 1 filters, filtered data, Alg. 2) ----
    def tomo_sirt_filters(self, geom, iters, filters, stream=None):
        n, na, nd = self.geoms[geom]
        self._check(self.lib.tomo_sirt_filters(
            self.h, geom, int(iters), _ptr(filters, (iters, na, nd), "filters"), _stream(stream)))

    def tomo_sirt_filter_sino(self, geom, filters, sino, out, stream=None):
        n, na, nd = self.geoms[geom]
        cnt = int(filters.shape[0]) if filters is not None and filters.dim() == 3 else 0
        self._check(self.lib.tomo_sirt_filter_sino(
            self.h, geom, _ptr(filters, (cnt, na, nd), "filters"), cnt,
            _ptr(sino, (na, nd), "sino"), _ptr(out, (cnt, na, nd), "out"), _stream(stream)))

    def roi_solve_local(self, geom, filtered, params, outs, stream=None):
        n, na, nd = self.geoms[geom]
        planes = int(filtered.shape[0]) if filtered is not None and filtered.dim() == 3 else 0
        cnt = len(params)
        parr = (roi_params * cnt)(*params)
        oarr = (C.c_void_p * cnt)(*[_ptr(o, (p.roi.rows, p.roi.cols), "out").value
                                    for o, p in zip(outs, params)])
        self._check(self.lib.roi_solve_local(self.h, geom, _ptr(filtered, (planes, na, nd),
                                                                "filtered"),
                                             planes, cnt, parr, oarr, _stream(stream)))

    # -- preprocessing of the local method ------------------------------------
    def tomo_disc_subtract(self, geom, sino, out, value, stream=None):
        n, na, nd = self.geoms[geom]
        self._check(self.lib.tomo_disc_subtract(
            self.h, geom, _ptr(sino, (na, nd), "sino"), _ptr(out, (na, nd), "out"),
            _ptr(value, (1,), "value"), _stream(stream)))

    def tomo_disc_add(self, geom, region, value, img, stream=None):
        r = _rect(region)
        self._check(self.lib.tomo_disc_add(self.h, geom, r, _ptr(value, (1,), "value"),
                                           _ptr(img, (r.rows, r.cols), "img"), _stream(stream)))

    def tomo_pad_truncated(self, geom, trunc, first_bin, out, stream=None):
        n, na, nd = self.geoms[geom]
        nb = int(trunc.shape[1]) if trunc is not None and trunc.dim() == 2 else 0
        self._check(self.lib.tomo_pad_truncated(
            self.h, geom, _ptr(trunc, (na, nb), "trunc"), int(first_bin), nb,
            _ptr(out, (na, nd), "out"), _stream(stream)))

    def roi_step_size(self, geom, ext):
        v = C.c_float()
        self._check(self.lib.roi_step_size(self.h, geom, _rect(ext), C.byref(v)))
        return v.value

    # -- serving --------------------------------------------------------
    def tomo_register_sinogram(self, geom, sino):
        n, na, nd = self.geoms[geom]
        sid = C.c_int32()
        self._check(self.lib.tomo_register_sinogram(
            self.h, geom, _ptr(sino, (na, nd), "sino", self.fake), C.byref(sid)))
        return sid.value

    def tomo_unregister_sinogram(self, sino_id):
        self._check(self.lib.tomo_unregister_sinogram(self.h, int(sino_id)))

    def roi_submit(self, sino_id, params, out):
        t = C.c_uint64()
        p = params
        st = self.lib.roi_submit(self.h, int(sino_id), C.byref(p),
                                 _ptr(out, (p.roi.rows, p.roi.cols), "out", self.fake),
                                 C.byref(t))
        self._check(st)
        return t.value

    def roi_poll(self, ticket):
        done = C.c_int()
        lat = C.c_float()
        self._check(self.lib.roi_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(lat)))
        return bool(done.value), (lat.value if done.value else None)

    def roi_poll_stages(self, ticket):
        """(done, None) or (True, dict(queued_ms, prepare_ms, run_ms, latency_ms))."""
        done = C.c_int()
        st = (C.c_float * 4)()
        self._check(self.lib.roi_poll_stages(self.h, C.c_uint64(ticket), C.byref(done), st))
        if not done.value:
            return False, None
        return True, dict(zip(("queued_ms", "prepare_ms", "run_ms", "latency_ms"), list(st)))

    def tomo_serving_fake(self, budget_bytes=0, tick_us=0):
        """Host test executor of serving (host-only context): budget_bytes > 0 sets it
        up; later calls with budget_bytes = 0 change tick_us (< 0 stalls)."""
        self._check(self.lib.tomo_serving_fake(self.h, C.c_size_t(int(budget_bytes)),
                                               int(tick_us)))
        self.fake = True

    def tomo_serving_config(self, max_slots=0, iters_per_tick=0):
        self._check(self.lib.tomo_serving_config(self.h, int(max_slots), int(iters_per_tick)))

    def tomo_set_launch(self, fp_segments=0, fp_rays_per_lane=0, fp_xcd_order=0, bp_variant=0,
                        bp_groups=0, bp_pixels_per_thread=0, bp_xcd_order=0):
        k = tomo_launch(int(fp_segments), int(fp_rays_per_lane), int(fp_xcd_order),
                        int(bp_variant), int(bp_groups), int(bp_pixels_per_thread),
                        int(bp_xcd_order))
        self._check(self.lib.tomo_set_launch(self.h, C.byref(k)))

    def tomo_get_launch(self):
        k = tomo_launch()
        self._check(self.lib.tomo_get_launch(self.h, C.byref(k)))
        return {f: getattr(k, f) for f, _ in tomo_launch._fields_}

    def tomo_resolve_launch(self, geom, params):
        """The launch shape a solve of this batch of parameters would use now."""
        cnt = len(params)
        parr = (roi_params * cnt)(*params)
        k = tomo_launch()
        self._check(self.lib.tomo_resolve_launch(self.h, geom, cnt, parr, C.byref(k)))
        return {f: getattr(k, f) for f, _ in tomo_launch._fields_}

    def tomo_autotune(self, geom, sino, params, outs, x_ext=None, stream=None):
        """Time every launch shape on this batch; returns (shape dict, fp_ms, bp_ms)."""
        n, na, nd = self.geoms[geom]
        cnt = len(params)
        parr = (roi_params * cnt)(*params)
        oarr = (C.c_void_p * cnt)(*[_ptr(o, (p.roi.rows, p.roi.cols), "out").value
                                    for o, p in zip(outs, params)])
        best = tomo_launch()
        ms = (C.c_float * 2)()
        self._check(self.lib.tomo_autotune(self.h, geom, _ptr(sino, (na, nd), "sino"),
                                           _ptr(x_ext, (n, n), "x_ext"), cnt, parr, oarr,
                                           _stream(stream), C.byref(best), ms))
        return {f: getattr(best, f) for f, _ in tomo_launch._fields_}, ms[0], ms[1]

    def tomo_set_graphs(self, enable=True):
        self._check(self.lib.tomo_set_graphs(self.h, int(bool(enable))))

    def tomo_roi_nnz(self, geom, region):
        v = C.c_int64()
        self._check(self.lib.tomo_roi_nnz(self.h, geom, _rect(region), C.byref(v)))
        return v.value

    def tomo_kernel_timing(self, mode=1):
        self._check(self.lib.tomo_kernel_timing(self.h, int(mode)))

    def tomo_kernel_time(self, kernel, reset=False):
        n, ms = C.c_int64(), C.c_double()
        self._check(self.lib.tomo_kernel_time(self.h, int(kernel), C.byref(n), C.byref(ms),
                                              int(bool(reset))))
        return n.value, ms.value

    def tomo_valu_probe(self, blocks, iters, a, b, out, mode=0, stream=None):
        self._check(self.lib.tomo_valu_probe(self.h, int(blocks), int(iters), int(mode), float(a),
                                             float(b), _ptr(out, (int(blocks) * 256,), "out"),
                                             _stream(stream)))

    def tomo_workspace_usage(self):
        u, p = C.c_size_t(), C.c_size_t()
        self._check(self.lib.tomo_workspace_usage(self.h, C.byref(u), C.byref(p)))
        return u.value, p.value

    def tomo_synchronize(self):
        self._check(self.lib.tomo_synchronize(self.h))
