"""ctypes binding of the C ABI declared in include/oc.h.

Argument marshalling only: every step of the method runs in the HIP library
``liboc.so``.  Bulk inputs/outputs of compute calls are device tensors
(PyTorch is used for device memory and streams); registration takes host
arrays.  There is no CPU fallback: importing this module without the built
library raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OC_LIB selects another build of the library (the checked variant,
# liboc_checked.so, for the bounds-checked test runs)
LIB_PATH = os.environ.get("OC_LIB") or os.path.join(_HERE, "liboc.so")

OC_OK, OC_EINVAL, OC_ENOMEM, OC_EDEVICE, OC_ENOTFOUND, OC_EBUDGET, OC_EGEOM, OC_ECAPACITY = 0, -1, -2, -3, -4, -5, -6, -7
OC_ETIMEDOUT = -8
OC_ESTARTED = -9
OC_HOLE, OC_FIELD, OC_FRINGE = 0, 1, -1
OC_SURF_WALL, OC_SURF_OVERSET = 0, 1
OC_FACE_INTERIOR, OC_FACE_WALL, OC_FACE_OVERSET, OC_FACE_FARFIELD = 0, 1, 2, 3
OC_TUNE_SURF_BINS, OC_TUNE_EXACT_WAVES, OC_TUNE_SERVICE_SLOTS, OC_TUNE_HBM_BUDGET, OC_TUNE_DONOR_WAVES = 1, 2, 3, 4, 5
OC_TUNE_DONOR_PAIRS = 6
OC_TUNE_FILTER_BLOCK = 7
OC_TUNE_POINT_TILES = 8
OC_TUNE_SIDE_LIST = 9

EXPORTS = ["oc_create", "oc_destroy", "oc_last_error", "oc_set_stream", "oc_register_grid",
           "oc_register_cut_surface", "oc_cut", "oc_cut_multi", "oc_last_cut_info", "oc_fringe_points",
           "oc_donor_search", "oc_last_donor_info", "oc_timing", "oc_timing_report", "oc_memory_used",
           "oc_slot_create", "oc_slot_destroy", "oc_slot_set_stream", "oc_slot_bytes", "oc_slot_cut",
           "oc_slot_fringe_points", "oc_slot_donor_search", "oc_slot_cut_info", "oc_slot_donor_info",
           "oc_cut_warm", "oc_sweep_bound", "oc_slot_cut_warm", "oc_cut_batch", "oc_slot_cut_batch",
           "oc_slot_create_batch", "oc_tune", "oc_unblank", "oc_element_points", "oc_ab_faces", "oc_face_points",
           "oc_interp_weights", "oc_slot_ab_faces", "oc_slot_face_points", "oc_slot_interp_weights", "oc_cut_filtered", "oc_slot_unblank", "oc_slot_element_points",
           "oc_submit", "oc_wait", "oc_service_info", "oc_donor_search_noalloc", "oc_noalloc_max_points",
           "oc_cut_refined", "oc_cancel", "oc_cut_posed", "oc_slot_cut_posed", "oc_check_word"]


class OcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("oc status %d: %s" % (status, msg))
        self.status = status


class oc_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("surf_bins", C.c_int32), ("donor_bin_scale", C.c_double),
                ("hbm_budget", C.c_int64), ("tune_cache", C.c_char_p)]


class oc_cut_info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_elem", "n_inbox", "n_near", "n_far", "n_hit", "n_hole",
                                         "n_cand_pairs", "n_side")]


class oc_cut_req(C.Structure):
    _fields_ = [("grid_id", C.c_int32), ("n_surf", C.c_int32), ("surf_ids", C.POINTER(C.c_int32)),
                ("poses", C.c_void_p), ("iblank_out", C.c_void_p)]


class oc_service_stats(C.Structure):
    _fields_ = [("slots", C.c_int32), ("running", C.c_int32), ("queued", C.c_int32), ("finished", C.c_int32),
                ("peak_running", C.c_int32), ("pad", C.c_int32), ("slot_bytes", C.c_int64)]


class oc_donor_info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_points", "n_newton", "n_iter", "n_orphan", "n_overflow")]


_lib = None


def load(path=LIB_PATH):
    """Load liboc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("HIP library %s is missing: build it with paper_1711_07663_amd/build.py "
                          "(no CPU fallback exists)" % path)
    L = C.CDLL(path)
    vp, dp, i32p, i8p, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p, C.POINTER(C.c_int64)
    sig = {
        "oc_create": ([C.POINTER(C.c_void_p), C.POINTER(oc_config)]),
        "oc_destroy": ([vp]),
        "oc_set_stream": ([vp, vp]),
        "oc_register_grid": ([vp, dp, C.c_int64, i32p, C.c_int64, C.POINTER(C.c_int8), i32p]),
        "oc_register_cut_surface": ([vp, dp, C.c_int64, i32p, C.c_int64, C.c_int32, i32p]),
        "oc_cut": ([vp, C.c_int32, C.c_int32, dp, vp]),
        "oc_cut_multi": ([vp, C.c_int32, i32p, dp, C.c_int32, vp]),
        "oc_last_cut_info": ([vp, C.POINTER(oc_cut_info)]),
        "oc_fringe_points": ([vp, C.c_int32, dp, vp, vp, C.c_int64, i64p, vp]),
        "oc_donor_search": ([vp, C.c_int32, dp, vp, C.c_int64, vp, vp]),
        "oc_donor_search_noalloc": ([vp, C.c_int32, dp, vp, C.c_int64, vp, vp]),
        "oc_noalloc_max_points": ([i64p]),
        "oc_last_donor_info": ([vp, C.POINTER(oc_donor_info)]),
        "oc_timing": ([vp, C.c_int32]),
        "oc_timing_report": ([vp, C.c_char_p, C.c_int64]),
        "oc_memory_used": ([vp, i64p]),
        "oc_slot_create": ([vp, i32p, C.c_int32, i32p, C.c_int32, C.c_int64, C.POINTER(C.c_void_p)]),
        "oc_slot_destroy": ([vp]),
        "oc_slot_set_stream": ([vp, vp]),
        "oc_slot_bytes": ([vp, i64p]),
        "oc_slot_cut": ([vp, C.c_int32, i32p, vp, C.c_int32, vp]),
        "oc_slot_fringe_points": ([vp, C.c_int32, vp, vp, vp, C.c_int64, vp, vp]),
        "oc_slot_donor_search": ([vp, C.c_int32, vp, vp, C.c_int64, vp, vp, vp]),
        "oc_slot_cut_info": ([vp, C.POINTER(oc_cut_info)]),
        "oc_slot_donor_info": ([vp, C.POINTER(oc_donor_info)]),
        "oc_cut_warm": ([vp, C.c_int32, C.c_int32, dp, dp, vp, vp]),
        "oc_sweep_bound": ([vp, C.c_int32, dp, dp, dp]),
        "oc_slot_cut_warm": ([vp, C.c_int32, C.c_int32, vp, C.c_double, vp, vp]),
        "oc_cut_batch": ([vp, C.POINTER(oc_cut_req), C.c_int32]),
        "oc_slot_cut_batch": ([vp, C.POINTER(oc_cut_req), C.c_int32]),
        "oc_slot_create_batch": ([vp, C.POINTER(oc_cut_req), C.c_int32, C.c_int64, C.POINTER(C.c_void_p)]),
        "oc_tune": ([vp, C.c_int32, C.c_int32, C.c_int64, i64p]),
        "oc_submit": ([vp, C.POINTER(oc_cut_req), C.POINTER(C.c_uint64)]),
        "oc_wait": ([vp, C.c_uint64, C.c_int32]),
        "oc_cancel": ([vp, C.c_uint64]),
        "oc_check_word": ([vp, C.POINTER(C.c_uint32), C.c_int32, C.POINTER(C.c_int32)]),
        "oc_cut_posed": ([vp, C.c_int32, dp, i32p, dp, C.c_int32, vp]),
        "oc_slot_cut_posed": ([vp, C.c_int32, vp, i32p, vp, C.c_int32, vp]),
        "oc_service_info": ([vp, C.POINTER(oc_service_stats)]),
        "oc_unblank": ([vp, C.c_int32, i32p, C.c_int32, dp, dp, vp, vp, vp, C.c_int64, i64p]),
        "oc_element_points": ([vp, C.c_int32, dp, vp, C.c_int64, vp, vp]),
        "oc_ab_faces": ([vp, C.c_int32, vp, vp, C.c_int64, i64p]),
        "oc_face_points": ([vp, C.c_int32, dp, vp, C.c_int64, dp, C.c_int32, vp, vp]),
        "oc_interp_weights": ([vp, vp, vp, C.c_int64, dp, C.c_int32, vp]),
        "oc_slot_ab_faces": ([vp, C.c_int32, vp, vp, C.c_int64, vp]),
        "oc_slot_face_points": ([vp, C.c_int32, vp, vp, vp, C.c_int64, dp, C.c_int32, vp, C.c_int64, vp, vp]),
        "oc_slot_interp_weights": ([vp, vp, vp, vp, C.c_int64, dp, C.c_int32, vp]),
        "oc_cut_filtered": ([vp, C.c_int32, i32p, dp, C.c_int32, C.c_int32, C.c_int32, vp, i64p]),
        "oc_cut_refined": ([vp, C.c_int32, i32p, dp, C.c_int32, C.c_int32, vp, i64p]),
        "oc_slot_unblank": ([vp, C.c_int32, i32p, C.c_int32, vp, vp, vp, vp, C.c_int64, vp]),
        "oc_slot_element_points": ([vp, C.c_int32, vp, vp, vp, C.c_int64, vp, vp, vp]),
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    L.oc_last_error.argtypes = []
    L.oc_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(st):
    if st != OC_OK:
        raise OcError(st, load().oc_last_error().decode())


def _pose(p):
    a = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


GAUSS3 = (-0.7745966692414834, 0.0, 0.7745966692414834)   # 3-point Gauss-Legendre nodes, +-sqrt(3/5)


def _nodes1d(z):
    a = np.ascontiguousarray(z, dtype=np.float64).reshape(-1)
    return a, a.ctypes.data_as(C.POINTER(C.c_double)), a.size


def _dptr(t, dtype, n=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
        raise TypeError("expected a contiguous %s CUDA tensor" % dtype)
    if n is not None and t.numel() < n:
        raise ValueError("tensor too small: %d < %d" % (t.numel(), n))
    return C.c_void_p(t.data_ptr())


_NP = {"int8": np.int8, "int32": np.int32, "float64": np.float64}


def _aptr(t, dtype, n=None):
    """Pointer of a contiguous array in host or device memory: a torch
    tensor (CUDA or CPU) or a numpy array of the given dtype (the library
    tells the two memories apart by the pointer)."""
    import torch
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous() or t.dtype != dtype:
            raise TypeError("expected a contiguous %s tensor" % dtype)
        if n is not None and t.numel() < n:
            raise ValueError("tensor too small: %d < %d" % (t.numel(), n))
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        want = _NP[str(dtype).replace("torch.", "")]
        if not t.flags.c_contiguous or t.dtype != want:
            raise TypeError("expected a C-contiguous %s array" % np.dtype(want).name)
        if n is not None and t.size < n:
            raise ValueError("array too small: %d < %d" % (t.size, n))
        return C.c_void_p(t.ctypes.data)
    raise TypeError("expected a torch tensor or a numpy array")


def _cut_reqs(ctx, reqs, device_poses):
    """oc_cut_req array for [(grid_id, surf_ids, poses, iblank)]; poses are
    host arrays [k,12] or, with device_poses, float64 CUDA tensors [k,12]
    (iblank may be None when only the shape of the batch matters).  Returns
    the array and the host buffers it points into (keep them alive)."""
    import torch
    arr = (oc_cut_req * max(len(reqs), 1))()
    keep = []
    for r, (gid, sids, poses, ib) in enumerate(reqs):
        ids = np.ascontiguousarray(sids, dtype=np.int32)
        keep.append(ids)
        arr[r].grid_id = int(gid)
        arr[r].n_surf = len(ids)
        arr[r].surf_ids = ids.ctypes.data_as(C.POINTER(C.c_int32))
        if len(ids) and poses is not None:
            if device_poses:
                arr[r].poses = _dptr(poses, torch.float64, 12 * len(ids)).value
            else:
                pa = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1)
                if pa.size != 12 * len(ids):
                    raise ValueError("request %d: %d poses for %d surfaces" % (r, pa.size // 12, len(ids)))
                keep.append(pa)
                arr[r].poses = pa.ctypes.data
        if ib is not None:
            arr[r].iblank_out = _dptr(ib, torch.int8, ctx.grids[gid]).value
    return arr, keep


class Context:
    """Owns one oc_ctx on one device; all compute calls run on ``stream``
    (torch's current stream of that device when not given)."""

    def __init__(self, device=0, surf_bins=0, donor_bin_scale=0.0, hbm_budget=0, stream=None, tune_cache=None):
        """tune_cache: path of a tuning file (autotune.save) applied at
        creation."""
        L = load()
        cfg = oc_config(device, surf_bins, donor_bin_scale, hbm_budget,
                        None if tune_cache is None else os.fsencode(tune_cache))
        h = C.c_void_p()
        _check(L.oc_create(C.byref(h), C.byref(cfg)))
        self._h = h
        self.device = device
        self._slots = weakref.WeakSet()
        self.grids = {}
        self.surfs = {}
        self.set_stream(stream)

    def close(self):
        """Destroy the context.  Its slots are destroyed with it: Slot
        objects still alive become closed handles."""
        if getattr(self, "_h", None):
            for sl in list(self._slots):
                sl._h = None
            self._slots.clear()
            load().oc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self.stream = stream
        _check(load().oc_set_stream(self._h, C.c_void_p(handle)))

    # -------------------------------------------------------- registration --
    @staticmethod
    def _reg_array(a, np_dtype, torch_dtype, width):
        """(pointer, rows, keep-alive) of a registration array: a torch
        tensor (CUDA or CPU, used in place) or anything numpy takes."""
        import torch
        if isinstance(a, torch.Tensor):
            a = a.contiguous().to(torch_dtype)
            if a.is_cuda:
                torch.cuda.synchronize(a.device)   # written by torch on its own streams
            return C.c_void_p(a.data_ptr()), a.numel() // width, a
        a = np.ascontiguousarray(a, dtype=np_dtype)
        return C.c_void_p(a.ctypes.data), a.size // width, a

    def register_grid(self, nodes, conn, face_tags=None):
        """nodes [n,3] FP64, conn [e,27] int32, face_tags [e,6] int8 (may be
        None): numpy arrays or torch tensors in host or device memory."""
        import torch
        pn, n_nodes, kn = self._reg_array(nodes, np.float64, torch.float64, 3)
        pc, n_elem, kc = self._reg_array(conn, np.int32, torch.int32, 27)
        pt, kt = None, None
        if face_tags is not None:
            pt, _, kt = self._reg_array(face_tags, np.int8, torch.int8, 6)
        gid = C.c_int32(-1)
        _check(load().oc_register_grid(self._h, C.cast(pn, C.POINTER(C.c_double)), n_nodes,
                                       C.cast(pc, C.POINTER(C.c_int32)), n_elem,
                                       None if pt is None else C.cast(pt, C.POINTER(C.c_int8)), C.byref(gid)))
        self.grids[gid.value] = int(n_elem)
        return gid.value

    def register_cut_surface(self, nodes, conn, kind=OC_SURF_WALL):
        """nodes [n,3] FP64, conn [f,9] int32: numpy arrays or torch tensors
        in host or device memory."""
        import torch
        pn, n_nodes, kn = self._reg_array(nodes, np.float64, torch.float64, 3)
        pc, n_face, kc = self._reg_array(conn, np.int32, torch.int32, 9)
        sid = C.c_int32(-1)
        _check(load().oc_register_cut_surface(self._h, C.cast(pn, C.POINTER(C.c_double)), n_nodes,
                                              C.cast(pc, C.POINTER(C.c_int32)), n_face, int(kind), C.byref(sid)))
        self.surfs[sid.value] = int(n_face)
        return sid.value

    # -------------------------------------------------------------- compute --
    def cut(self, grid_id, surf_id, pose, iblank):
        """iblank: int8 tensor (CUDA or CPU) or numpy array."""
        import torch
        _, pp = _pose(pose)
        _check(load().oc_cut(self._h, grid_id, surf_id, pp, _aptr(iblank, torch.int8, self.grids[grid_id])))
        return iblank

    def cut_multi(self, grid_id, surf_ids, poses, iblank):
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        pa, pp = _pose(np.asarray(poses, dtype=np.float64).reshape(-1) if len(ids) else np.zeros(12))
        _check(load().oc_cut_multi(self._h, grid_id, ids.ctypes.data_as(C.POINTER(C.c_int32)), pp, len(ids),
                                   _aptr(iblank, torch.int8, self.grids[grid_id])))
        return iblank

    def cut_posed(self, grid_id, grid_pose, surf_ids, poses, iblank):
        """oc_cut_posed: grid and surfaces at world-frame poses (host)."""
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        _, gp = _pose(grid_pose)
        pa, pp = _pose(np.asarray(poses, dtype=np.float64).reshape(-1) if len(ids) else np.zeros(12))
        _check(load().oc_cut_posed(self._h, grid_id, gp, ids.ctypes.data_as(C.POINTER(C.c_int32)), pp, len(ids),
                                   _aptr(iblank, torch.int8, self.grids[grid_id])))
        return iblank

    def cut_batch(self, reqs):
        """reqs: [(grid_id, surf_ids, host poses [k,12], iblank tensor)];
        every request's cuts in one launch per stage."""
        arr, keep = _cut_reqs(self, reqs, device_poses=False)
        _check(load().oc_cut_batch(self._h, arr, len(reqs)))

    def submit(self, grid_id, surf_ids, poses, iblank):
        """Queue one cut request (host poses [k,12], iblank tensor) on the
        cut service; returns its ticket at once."""
        arr, keep = _cut_reqs(self, [(grid_id, surf_ids, poses, iblank)], device_poses=False)
        t = C.c_uint64(0)
        _check(load().oc_submit(self._h, arr, C.byref(t)))
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        """True once the request has finished (its iblank is written),
        False if timeout_ms passed first; raises the request's failure."""
        st = load().oc_wait(self._h, C.c_uint64(ticket), int(timeout_ms))
        if st == OC_ETIMEDOUT:
            return False
        _check(st)
        return True

    def check_word(self, clear=False):
        """(word, checked): the bounds-check word of a checked build
        (liboc_checked.so) and whether this library is one."""
        w, c = C.c_uint32(0), C.c_int32(0)
        _check(load().oc_check_word(self._h, C.byref(w), int(bool(clear)), C.byref(c)))
        return w.value, bool(c.value)

    def cancel(self, ticket):
        """Drop a request that is still queued (True); False when it has
        already started or finished (retire it with wait)."""
        st = load().oc_cancel(self._h, C.c_uint64(ticket))
        if st == OC_ESTARTED:
            return False
        _check(st)
        return True

    def service_info(self):
        v = oc_service_stats()
        _check(load().oc_service_info(self._h, C.byref(v)))
        return {n: getattr(v, n) for n, _ in oc_service_stats._fields_ if n != "pad"}

    def cut_warm(self, grid_id, surf_id, pose, prev_pose, prev_iblank, iblank):
        import torch
        _, pp = _pose(pose)
        _, qq = _pose(prev_pose)
        _check(load().oc_cut_warm(self._h, grid_id, surf_id, pp, qq, _dptr(prev_iblank, torch.int8, self.grids[grid_id]),
                                  _dptr(iblank, torch.int8, self.grids[grid_id])))
        return iblank

    def unblank(self, grid_id, surf_ids, poses_t, poses_tp, prev_iblank, iblank, unblank_out):
        """Blanking of a moving grid's time step with unblanking (oc_unblank);
        returns the number of cells to unblank (their ids in unblank_out)."""
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        n = len(ids)
        pa, pp = _pose(np.asarray(poses_t, dtype=np.float64).reshape(-1) if n else np.zeros(12))
        qa, qq = _pose(np.asarray(poses_tp, dtype=np.float64).reshape(-1) if n else np.zeros(12))
        cnt = C.c_int64(0)
        ne = self.grids[grid_id]
        _check(load().oc_unblank(self._h, grid_id, ids.ctypes.data_as(C.POINTER(C.c_int32)), n, pp, qq,
                                 _dptr(prev_iblank, torch.int8, ne), _dptr(iblank, torch.int8, ne),
                                 _dptr(unblank_out, torch.int32), unblank_out.numel(), C.byref(cnt)))
        return cnt.value

    def element_points(self, grid_id, pose, elems, n, points, src=None):
        """27 Gauss points of each of the first n element ids of ``elems``."""
        import torch
        _, pp = _pose(pose)
        if n == 0:
            return
        _check(load().oc_element_points(self._h, grid_id, pp, _dptr(elems, torch.int32, n), int(n),
                                        _dptr(points, torch.float64, 81 * n),
                                        None if src is None else _dptr(src, torch.int32, 27 * n)))

    def cut_filtered(self, grid_id, surf_ids, poses, iblank, nf1=16, nf2=4):
        """The paper's filtered cut (oc_cut_filtered); returns the number of
        (surface, element) pairs it examined."""
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        pa, pp = _pose(np.asarray(poses, dtype=np.float64).reshape(-1) if len(ids) else np.zeros(12))
        n = C.c_int64(0)
        _check(load().oc_cut_filtered(self._h, grid_id, ids.ctypes.data_as(C.POINTER(C.c_int32)), pp, len(ids),
                                      int(nf1), int(nf2), _dptr(iblank, torch.int8, self.grids[grid_id]), C.byref(n)))
        return n.value

    def cut_refined(self, grid_id, surf_ids, poses, iblank, k):
        """The cut with the curved faces resolved to level k
        (oc_cut_refined); returns the number of (surface, element) items
        refined."""
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        pa, pp = _pose(np.asarray(poses, dtype=np.float64).reshape(-1))
        n = C.c_int64(0)
        _check(load().oc_cut_refined(self._h, grid_id, ids.ctypes.data_as(C.POINTER(C.c_int32)), pp, len(ids),
                                     int(k), _dptr(iblank, torch.int8, self.grids[grid_id]), C.byref(n)))
        return n.value

    def ab_faces(self, grid_id, iblank, faces):
        """Artificial-boundary faces (ids 6 e + f, ascending) into ``faces``
        (int32 device tensor); returns their number."""
        import torch
        n = C.c_int64(0)
        _check(load().oc_ab_faces(self._h, grid_id, _dptr(iblank, torch.int8, self.grids[grid_id]),
                                  _dptr(faces, torch.int32), faces.numel(), C.byref(n)))
        return n.value

    def face_points(self, grid_id, pose, faces, n, points, src=None, nodes1d=GAUSS3):
        """m x m flux points per face id of the first n entries of ``faces``."""
        import torch
        _, pp = _pose(pose)
        z, zp, m = _nodes1d(nodes1d)
        if n == 0:
            return
        _check(load().oc_face_points(self._h, grid_id, pp, _dptr(faces, torch.int32, n), int(n), zp, m,
                                     _dptr(points, torch.float64, 3 * m * m * n),
                                     None if src is None else _dptr(src, torch.int32, m * m * n)))

    def interp_weights(self, donors, ref, n, weights, nodes1d=GAUSS3):
        """m^3 Lagrange weights per receptor (NaN for orphans)."""
        import torch
        z, zp, m = _nodes1d(nodes1d)
        if n == 0:
            return
        _check(load().oc_interp_weights(self._h, _dptr(donors, torch.int32, n), _dptr(ref, torch.float64, 3 * n),
                                        int(n), zp, m, _dptr(weights, torch.float64, n * m ** 3)))

    def sweep_bound(self, surf_id, pose_a, pose_b):
        _, pa = _pose(pose_a)
        _, pb = _pose(pose_b)
        v = C.c_double(0)
        _check(load().oc_sweep_bound(self._h, surf_id, pa, pb, C.byref(v)))
        return v.value

    def last_cut_info(self):
        info = oc_cut_info()
        _check(load().oc_last_cut_info(self._h, C.byref(info)))
        return {n: getattr(info, n) for n, _ in oc_cut_info._fields_}

    def last_donor_info(self):
        info = oc_donor_info()
        _check(load().oc_last_donor_info(self._h, C.byref(info)))
        return {n: getattr(info, n) for n, _ in oc_donor_info._fields_}

    def fringe_points(self, grid_id, pose, iblank, points, src=None):
        """Fills ``points`` (float64 [cap,3]) and ``src`` (int32 [cap]);
        returns the number of points written."""
        import torch
        _, pp = _pose(pose)
        n = C.c_int64(0)
        cap = (points.numel() if isinstance(points, torch.Tensor) else points.size) // 3
        _check(load().oc_fringe_points(self._h, grid_id, pp, _aptr(iblank, torch.int8, self.grids[grid_id]),
                                       _aptr(points, torch.float64), cap, C.byref(n),
                                       None if src is None else _aptr(src, torch.int32, cap)))
        return n.value

    def donor_search(self, grid_id, pose, points, n, donor, ref):
        import torch
        _, pp = _pose(pose)
        if n == 0:
            return
        _check(load().oc_donor_search(self._h, grid_id, pp, _aptr(points, torch.float64, 3 * n), int(n),
                                      _aptr(donor, torch.int32, n), _aptr(ref, torch.float64, 3 * n)))

    def donor_search_noalloc(self, grid_id, pose, points, n, donor, ref):
        """oc_donor_search_noalloc: the donor search on the library's fixed
        scratch array (no allocation; at most noalloc_max_points() points)."""
        import torch
        _, pp = _pose(pose)
        _check(load().oc_donor_search_noalloc(self._h, grid_id, pp,
                                              _dptr(points, torch.float64, 3 * n) if n else None, int(n),
                                              _dptr(donor, torch.int32, n) if n else None,
                                              _dptr(ref, torch.float64, 3 * n) if n else None))

    @staticmethod
    def noalloc_max_points():
        v = C.c_int64(0)
        _check(load().oc_noalloc_max_points(C.byref(v)))
        return v.value

    # ------------------------------------------------------------- timing ---
    def timing(self, enable):
        _check(load().oc_timing(self._h, 1 if enable else 0))

    def timing_report(self):
        buf = C.create_string_buffer(1 << 16)
        _check(load().oc_timing_report(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def tune(self, knob, arg, value):
        """Set a tuning knob (OC_TUNE_*); returns the value in force."""
        v = C.c_int64(0)
        _check(load().oc_tune(self._h, int(knob), int(arg), int(value), C.byref(v)))
        return v.value

    def memory_used(self):
        v = C.c_int64(0)
        _check(load().oc_memory_used(self._h, C.byref(v)))
        return v.value

    def create_slot(self, grid_ids, surf_ids, points_cap=0, stream=None):
        return Slot(self, grid_ids, surf_ids, points_cap, stream)

    def create_batch_slot(self, reqs, points_cap=0, stream=None):
        """Slot sized for batches shaped like reqs [(grid_id, surf_ids, ...)]."""
        return Slot(self, None, None, points_cap, stream, batch=[(r[0], r[1], None, None) for r in reqs])


def _dev_or_null(t, dtype):
    return None if t is None else _dptr(t, dtype)


class Slot:
    """Per-request scratch reserved up front (oc_slot_create).  Its calls
    take device poses (float64 [k,12] tensors) and device point counts
    (int32 tensors), never allocate and never synchronise, so they can be
    captured in a graph or run concurrently with other slots."""

    def __init__(self, ctx: Context, grid_ids, surf_ids, points_cap=0, stream=None, batch=None):
        import torch
        self.ctx = ctx
        h = C.c_void_p()
        if batch is not None:
            arr, keep = _cut_reqs(ctx, batch, device_poses=True)
            _check(load().oc_slot_create_batch(ctx._h, arr, len(batch), int(points_cap), C.byref(h)))
        else:
            g = np.ascontiguousarray(grid_ids, dtype=np.int32)
            sid = np.ascontiguousarray(surf_ids, dtype=np.int32)
            _check(load().oc_slot_create(ctx._h, g.ctypes.data_as(C.POINTER(C.c_int32)), len(g),
                                         sid.ctypes.data_as(C.POINTER(C.c_int32)), len(sid), int(points_cap),
                                         C.byref(h)))
        self._h = h
        ctx._slots.add(self)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=ctx.device)
        self.set_stream(self.stream)

    def close(self):
        if getattr(self, "_h", None):
            load().oc_slot_destroy(self._h)
            self._h = None
            self.ctx._slots.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(load().oc_slot_set_stream(self._h, C.c_void_p(handle)))

    def nbytes(self):
        v = C.c_int64(0)
        _check(load().oc_slot_bytes(self._h, C.byref(v)))
        return v.value

    def cut(self, grid_id, surf_ids, poses_dev, iblank):
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        pp = _dptr(poses_dev, torch.float64, 12 * len(ids)) if len(ids) else None
        _check(load().oc_slot_cut(self._h, grid_id, ids.ctypes.data_as(C.POINTER(C.c_int32)), pp, len(ids),
                                  _dptr(iblank, torch.int8, self.ctx.grids[grid_id])))

    def cut_posed(self, grid_id, grid_pose_dev, surf_ids, poses_dev, iblank):
        """oc_slot_cut_posed: world-frame device poses (grid [12], surfaces
        [k,12]), composed on the slot stream."""
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        pp = _dptr(poses_dev, torch.float64, 12 * len(ids)) if len(ids) else None
        _check(load().oc_slot_cut_posed(self._h, grid_id, _dptr(grid_pose_dev, torch.float64, 12),
                                        ids.ctypes.data_as(C.POINTER(C.c_int32)), pp, len(ids),
                                        _dptr(iblank, torch.int8, self.ctx.grids[grid_id])))

    def cut_batch(self, reqs):
        """reqs: [(grid_id, surf_ids, device poses [k,12] tensor, iblank)]."""
        arr, keep = _cut_reqs(self.ctx, reqs, device_poses=True)
        _check(load().oc_slot_cut_batch(self._h, arr, len(reqs)))

    def cut_warm(self, grid_id, surf_id, pose_dev, sweep, prev_iblank, iblank):
        import torch
        _check(load().oc_slot_cut_warm(self._h, grid_id, surf_id, _dptr(pose_dev, torch.float64, 12), float(sweep),
                                       _dptr(prev_iblank, torch.int8, self.ctx.grids[grid_id]),
                                       _dptr(iblank, torch.int8, self.ctx.grids[grid_id])))

    def fringe_points(self, grid_id, pose_dev, iblank, points, n_dev, src=None):
        import torch
        cap = points.numel() // 3
        _check(load().oc_slot_fringe_points(self._h, grid_id, _dptr(pose_dev, torch.float64, 12),
                                            _dptr(iblank, torch.int8), _dptr(points, torch.float64), cap,
                                            _dptr(n_dev, torch.int32, 1),
                                            None if src is None else _dptr(src, torch.int32, cap)))

    def donor_search(self, grid_id, pose_dev, points, cap, n_dev, donor, ref):
        import torch
        _check(load().oc_slot_donor_search(self._h, grid_id, _dptr(pose_dev, torch.float64, 12),
                                           _dptr(points, torch.float64, 3 * cap), int(cap),
                                           _dev_or_null(n_dev, torch.int32), _dptr(donor, torch.int32, cap),
                                           _dptr(ref, torch.float64, 3 * cap)))

    def unblank(self, grid_id, surf_ids, poses_dev, prev_iblank, iblank, unblank_out, n_dev):
        """poses_dev: float64 [2k, 12] device tensor (poses of t, then of t + dt)."""
        import torch
        ids = np.ascontiguousarray(surf_ids, dtype=np.int32)
        ne = self.ctx.grids[grid_id]
        _check(load().oc_slot_unblank(self._h, grid_id, ids.ctypes.data_as(C.POINTER(C.c_int32)), len(ids),
                                      _dptr(poses_dev, torch.float64, 24 * len(ids)) if len(ids) else None,
                                      _dptr(prev_iblank, torch.int8, ne), _dptr(iblank, torch.int8, ne),
                                      _dptr(unblank_out, torch.int32), unblank_out.numel(),
                                      _dptr(n_dev, torch.int32, 1)))

    def element_points(self, grid_id, pose_dev, elems, n_dev, points, n_points_dev=None, src=None):
        import torch
        cap = points.numel() // 3
        _check(load().oc_slot_element_points(self._h, grid_id, _dptr(pose_dev, torch.float64, 12),
                                             _dptr(elems, torch.int32), _dptr(n_dev, torch.int32, 1), cap,
                                             _dptr(points, torch.float64), _dev_or_null(n_points_dev, torch.int32),
                                             None if src is None else _dptr(src, torch.int32, cap)))

    def ab_faces(self, grid_id, iblank, faces, n_dev):
        import torch
        _check(load().oc_slot_ab_faces(self._h, grid_id, _dptr(iblank, torch.int8, self.ctx.grids[grid_id]),
                                       _dptr(faces, torch.int32), faces.numel(), _dptr(n_dev, torch.int32, 1)))

    def face_points(self, grid_id, pose_dev, faces, n_faces_dev, points, n_dev, src=None, nodes1d=GAUSS3):
        import torch
        z, zp, m = _nodes1d(nodes1d)
        cap = points.numel() // 3
        _check(load().oc_slot_face_points(self._h, grid_id, _dptr(pose_dev, torch.float64, 12),
                                          _dptr(faces, torch.int32), _dev_or_null(n_faces_dev, torch.int32),
                                          faces.numel(), zp, m, _dptr(points, torch.float64), cap,
                                          _dev_or_null(n_dev, torch.int32),
                                          None if src is None else _dptr(src, torch.int32, cap)))

    def interp_weights(self, donors, ref, cap, n_dev, weights, nodes1d=GAUSS3):
        import torch
        z, zp, m = _nodes1d(nodes1d)
        _check(load().oc_slot_interp_weights(self._h, _dptr(donors, torch.int32, cap), _dptr(ref, torch.float64, 3 * cap),
                                             _dev_or_null(n_dev, torch.int32), int(cap), zp, m,
                                             _dptr(weights, torch.float64, cap * m ** 3)))

    def cut_info(self):
        info = oc_cut_info()
        _check(load().oc_slot_cut_info(self._h, C.byref(info)))
        return {n: getattr(info, n) for n, _ in oc_cut_info._fields_}

    def donor_info(self):
        info = oc_donor_info()
        _check(load().oc_slot_donor_info(self._h, C.byref(info)))
        return {n: getattr(info, n) for n, _ in oc_donor_info._fields_}
