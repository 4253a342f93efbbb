"""Python front end over the C ABI.  Torch provides device memory and streams only."""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np

from . import _lib
from ._lib import check



def _library_alive() -> bool:
    """False while the interpreter tears modules down: a handle collected then is left to
    the process exit instead of being freed through a half-cleared module."""
    return _lib is not None and callable(getattr(_lib, "lib", None))

def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return ctypes.c_void_p(t.ctypes.data)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Cloud:
    """A point cloud with its successor lists (built on the host, resident on the GPU)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @classmethod
    def build(cls, points: np.ndarray, order: Optional[np.ndarray] = None,
              device: bool = False, stream=None) -> "Cloud":
        """points: float32 [n,3] in caller order; order[r] = caller index of rank r.
        device=True builds the same lists on the GPU (mknn_build_device) on `stream`
        (a torch.cuda.Stream, default: torch's current stream)."""
        pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
        o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
        if o is not None and o.shape[0] != pts.shape[0]:
            raise ValueError("order must have one entry per point")
        h = ctypes.c_void_p()
        if device:
            check(_lib.lib().mknn_build_device(_ptr(pts), pts.shape[0], _ptr(o),
                                               _stream(stream), ctypes.byref(h)))
        else:
            check(_lib.lib().mknn_build(_ptr(pts), pts.shape[0], _ptr(o), ctypes.byref(h)))
        return cls(h)

    def __del__(self):
        if _library_alive():
            self.close()

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().mknn_free(self._h)
            self._h = None

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def n(self) -> int:
        return int(_lib.lib().mknn_size(self._h))

    def successors(self) -> Tuple[np.ndarray, np.ndarray]:
        """(offsets int64 [n+1], ranks int32 [nnz]) -- copies of the host CSR lists."""
        off = ctypes.c_void_p()
        ent = ctypes.c_void_p()
        nnz = ctypes.c_int64()
        check(_lib.lib().mknn_successors(self._h, ctypes.byref(off), ctypes.byref(ent),
                                         ctypes.byref(nnz)))
        n = self.n
        offs = np.ctypeslib.as_array(ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), (n + 1,)).copy()
        if nnz.value:
            ranks = np.ctypeslib.as_array(ctypes.cast(ent, ctypes.POINTER(ctypes.c_int32)),
                                          (nnz.value,)).copy()
        else:
            ranks = np.zeros(0, np.int32)
        return offs, ranks

    def lists(self):
        """Successor lists as a list of Python lists (small clouds)."""
        off, ent = self.successors()
        return [ent[off[i]:off[i + 1]].tolist() for i in range(self.n)]

    def points_by_rank(self) -> np.ndarray:
        p = ctypes.c_void_p()
        check(_lib.lib().mknn_points_by_rank(self._h, ctypes.byref(p)))
        return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_float)),
                                     (self.n, 3)).copy()

    def delete(self, ranks, stream=None) -> None:
        """Delete live ranks (Alg. 3); updates the device lists too when uploaded."""
        r = np.ascontiguousarray(np.asarray(ranks, dtype=np.int32).reshape(-1))
        st = None
        if self.device_bytes:
            st = _stream(stream)
        check(_lib.lib().mknn_delete(self._h, _ptr(r), r.shape[0], st))

    def delete_lazy(self, ranks, stream=None) -> None:
        """Mark live ranks as deleted on the device; queries filter them until flush()
        (or a call that needs the lists current) runs Alg. 3.  Needs an uploaded cloud."""
        r = np.ascontiguousarray(np.asarray(ranks, dtype=np.int32).reshape(-1))
        check(_lib.lib().mknn_delete_lazy(self._h, _ptr(r), r.shape[0], _stream(stream)))

    def flush(self, stream=None) -> None:
        """Apply the deletions marked by delete_lazy (Alg. 3, then the device delta)."""
        check(_lib.lib().mknn_delete_flush(self._h, _stream(stream)))

    @property
    def pending_deletes(self) -> int:
        return int(_lib.lib().mknn_pending_deletes(self._h))

    def insert(self, points, stream=None) -> range:
        """Append points (float32 [count, 3]) as the newest ranks; returns their ranks."""
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32).reshape(-1, 3))
        n0 = self.n
        st = None
        if self.device_bytes:
            st = _stream(stream)
        check(_lib.lib().mknn_insert(self._h, _ptr(pts), pts.shape[0], st))
        return range(n0, self.n)

    @property
    def live_count(self) -> int:
        return int(_lib.lib().mknn_live_count(self._h))

    @property
    def head(self) -> int:
        return int(_lib.lib().mknn_head(self._h))

    # ---- device side
    def upload(self, stream=None) -> "Cloud":
        check(_lib.lib().mknn_upload(self._h, _stream(stream)))
        return self

    def compact(self, stream=None) -> "Cloud":
        """Pack the device lists again, giving back the slack used by deletion deltas."""
        check(_lib.lib().mknn_compact(self._h, _stream(stream)))
        return self

    @property
    def device_bytes(self) -> int:
        return int(_lib.lib().mknn_device_bytes(self._h))

    def knn(self, q, k: int, m: Optional[int] = None, out=None, stream=None):
        """q: float32 [nq,3] CUDA tensor -> (idx int32 [nq,k], dist float32 [nq,k])."""
        import torch
        q = q.contiguous()
        nq = q.shape[0]
        m = self.n if m is None else int(m)
        if out is None:
            idx = torch.empty((nq, k), dtype=torch.int32, device=q.device)
            dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        else:
            idx, dist = out
        check(_lib.lib().mknn_knn(self._h, _ptr(q), nq, int(k), m, _ptr(idx), _ptr(dist),
                                  _stream(stream)))
        return idx, dist

    def knn_plane(self, q, k: int, m: Optional[int] = None, stream=None):
        """k-NN rows plus a plane fitted to each row's neighbours: (idx, dist, plane) with
        plane float32 [nq, 8] = centroid xyz, unit normal xyz, RMS residual, variation."""
        import torch
        q = q.contiguous()
        nq = q.shape[0]
        m = self.n if m is None else int(m)
        idx = torch.empty((nq, k), dtype=torch.int32, device=q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        plane = torch.empty((nq, 8), dtype=torch.float32, device=q.device)
        check(_lib.lib().mknn_knn_plane(self._h, _ptr(q), nq, int(k), m, _ptr(idx), _ptr(dist),
                                        _ptr(plane), _stream(stream)))
        return idx, dist, plane

    def knn_var(self, q, k_per_query, m_per_query, stream=None):
        """Per-query k and m; returns (idx, dist, row_off) with ragged rows (flat tensors)."""
        import torch
        q = q.contiguous()
        nq = q.shape[0]
        kq = k_per_query.to(torch.int32).contiguous()
        mq = m_per_query.to(torch.int32).contiguous()
        row_off = torch.zeros(nq + 1, dtype=torch.int64, device=q.device)
        if nq:
            torch.cumsum(kq.to(torch.int64), 0, out=row_off[1:])
        tot = int(row_off[-1].item()) if nq else 0
        kmax = int(kq.max().item()) if nq else 1
        idx = torch.empty(tot, dtype=torch.int32, device=q.device)
        dist = torch.empty(tot, dtype=torch.float32, device=q.device)
        check(_lib.lib().mknn_knn_var(self._h, _ptr(q), nq, _ptr(kq), _ptr(mq), _ptr(row_off),
                                      kmax, _ptr(idx), _ptr(dist), _stream(stream)))
        return idx, dist, row_off

    def knn_counts(self, q, k: int, m: Optional[int] = None, stream=None,
                   inserts: bool = False):
        """Per-query work: (entries examined E, lists opened L[, inserts]) as int32 tensors."""
        import torch
        q = q.contiguous()
        nq = q.shape[0]
        m = self.n if m is None else int(m)
        ce = torch.empty(nq, dtype=torch.int32, device=q.device)
        cl = torch.empty(nq, dtype=torch.int32, device=q.device)
        ci = torch.empty(nq, dtype=torch.int32, device=q.device) if inserts else None
        check(_lib.lib().mknn_knn_counts(self._h, _ptr(q), nq, int(k), m, _ptr(ce), _ptr(cl),
                                         _ptr(ci), _stream(stream)))
        return (ce, cl, ci) if inserts else (ce, cl)


FAMILIES = {1: "lane", 2: "group", 3: "rows"}


def autotune(cloud, q, k: int, m: Optional[int] = None, stream=None):
    """Time every kernel configuration on these queries and keep the fastest for clouds of
    this size class and this k class.  Returns (best, tried) as dicts."""
    tried = (_lib.TuneEntry * 16)()
    best = _lib.TuneEntry()
    n = ctypes.c_int32()
    q = q.contiguous()
    check(_lib.lib().mknn_autotune(cloud.handle, _ptr(q), q.shape[0], int(k),
                                   0 if m is None else int(m), _stream(stream), tried, 16,
                                   ctypes.byref(n), ctypes.byref(best)))

    def d(e):
        return {"family": FAMILIES[e.family], "merge_min": e.merge_min,
                "per_wave": e.per_wave, "ms": float(e.ms)}
    return d(best), [d(tried[i]) for i in range(min(n.value, 16))]


def tune_save(path: str) -> None:
    check(_lib.lib().mknn_tune_save(path.encode()))


def tune_load(path: str) -> None:
    check(_lib.lib().mknn_tune_load(path.encode()))


def tune_reset() -> None:
    _lib.lib().mknn_tune_reset()


def _requests(items):
    """items: sequence of (cloud, q, k, m, idx, dist) -> ctypes array of mknn_request."""
    arr = (_lib.Request * max(1, len(items)))()
    for i, (cloud, q, k, m, idx, dist) in enumerate(items):
        arr[i].cloud = cloud.handle.value
        arr[i].d_q = q.data_ptr() if q.numel() else None
        arr[i].nq = q.shape[0]
        arr[i].k = int(k)
        arr[i].m = 0 if m is None else int(m)
        arr[i].d_idx = idx.data_ptr() if idx.numel() else None
        arr[i].d_dist = dist.data_ptr() if dist.numel() else None
    return arr


def alloc_outputs(items):
    """items: (cloud, q, k, m) -> same plus freshly allocated (idx, dist) device tensors."""
    import torch
    out = []
    for cloud, q, k, m in items:
        idx = torch.empty((q.shape[0], k), dtype=torch.int32, device=q.device)
        dist = torch.empty((q.shape[0], k), dtype=torch.float32, device=q.device)
        out.append((cloud, q, k, m, idx, dist))
    return out


class BatchPlan:
    """Device buffers + captured hipGraph for batches of many clouds (mknn_batch_plan_*)."""

    def __init__(self, max_requests: int, max_queries: int, tile_queries: int = 16,
                 sort: bool = True, graph: bool = True):
        flags = (0 if sort else _lib.BATCH_NO_SORT) | (0 if graph else _lib.BATCH_NO_GRAPH)
        h = ctypes.c_void_p()
        check(_lib.lib().mknn_batch_plan_create(int(max_requests), int(max_queries),
                                                int(tile_queries), flags, ctypes.byref(h)))
        self._h = h

    def run(self, items, stream=None):
        """items: sequence of (cloud, q, k, m, idx, dist); enqueues the batch."""
        self._keep = _requests(items)
        check(_lib.lib().mknn_batch_plan_run(self._h, self._keep, len(items), _stream(stream)))

    def tune(self, items, stream=None) -> int:
        """Tune the plan's launch on batches like this one: the merge thresholds of the flat
        launch (returns the threshold of the class with most queries) or the tile length of
        the persistent launch (returns it)."""
        self._keep = _requests(items)
        t = ctypes.c_int32()
        check(_lib.lib().mknn_batch_plan_tune(self._h, self._keep, len(items), _stream(stream),
                                              ctypes.byref(t)))
        return t.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().mknn_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        if _library_alive():
            self.close()


def batch_knn(items, stream=None):
    """Convenience form of the batched call (library-owned plan)."""
    arr = _requests(items)
    check(_lib.lib().mknn_batch_knn(arr, len(items), _stream(stream)))


class Server:
    """Continuous-batching request loop (mknn_server_*).  Request buffers are torch tensors
    that must stay alive until the request completes; this wrapper keeps them until wait()."""

    def __init__(self, pool_queries: int = 1 << 21, nstreams: int = 2,
                 max_wave_requests: int = 256, plain: bool = False,
                 bind_at_admission: bool = False, lazy_delete: bool = False):
        flags = ((_lib.SERVER_PLAIN if plain else 0) |
                 (_lib.SERVER_BIND_AT_ADMISSION if bind_at_admission else 0) |
                 (_lib.SERVER_LAZY_DELETE if lazy_delete else 0))
        h = ctypes.c_void_p()
        check(_lib.lib().mknn_server_create(int(pool_queries), int(nstreams),
                                            int(max_wave_requests), flags, ctypes.byref(h)))
        self._h = h
        self._keep = {}

    @staticmethod
    def now() -> float:
        return float(_lib.lib().mknn_server_now())

    def submit(self, cloud, q, k: int, m=None, idx=None, dist=None, h_idx=None, h_dist=None):
        """Queue a request; returns its ticket.  Outputs are allocated when not given."""
        import torch
        if idx is None:
            idx = torch.empty((q.shape[0], k), dtype=torch.int32, device=q.device)
        if dist is None:
            dist = torch.empty((q.shape[0], k), dtype=torch.float32, device=q.device)
        req = _requests([(cloud, q, k, m, idx, dist)])
        t = ctypes.c_uint64()
        check(_lib.lib().mknn_server_submit(self._h, req, _ptr(h_idx), _ptr(h_dist),
                                            ctypes.byref(t)))
        self._keep[t.value] = (q, idx, dist, h_idx, h_dist)
        return t.value

    def delete(self, cloud, ranks):
        r = np.ascontiguousarray(np.asarray(ranks, dtype=np.int32).reshape(-1))
        t = ctypes.c_uint64()
        check(_lib.lib().mknn_server_delete(self._h, cloud.handle, _ptr(r), r.shape[0],
                                            ctypes.byref(t)))
        self._keep[t.value] = (r,)
        return t.value

    def insert(self, cloud, points):
        """Queue an insertion batch (float32 [count, 3]); ranks follow arrival order."""
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32).reshape(-1, 3))
        t = ctypes.c_uint64()
        check(_lib.lib().mknn_server_insert(self._h, cloud.handle, _ptr(pts), pts.shape[0],
                                            ctypes.byref(t)))
        self._keep[t.value] = (pts,)
        return t.value

    def done(self, ticket) -> bool:
        d = ctypes.c_int32()
        check(_lib.lib().mknn_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket, with_seen: bool = False):
        """Block until done; returns (submit_time, done_time, buffers[, updates_seen]):
        updates_seen counts the deletion and insertion batches a request saw."""
        t = (ctypes.c_double * 3)()
        v = ctypes.c_int64()
        st = _lib.lib().mknn_server_wait(self._h, ctypes.c_uint64(ticket), t, ctypes.byref(v))
        bufs = self._keep.pop(ticket, None)
        check(st)
        if with_seen:
            return t[0], t[2], bufs, v.value
        return t[0], t[2], bufs

    def stats(self):
        w, r = ctypes.c_int64(), ctypes.c_int64()
        check(_lib.lib().mknn_server_stats(self._h, ctypes.byref(w), ctypes.byref(r)))
        return w.value, r.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().mknn_server_destroy(self._h)
            self._h = None

    def __del__(self):
        if _library_alive():
            self.close()


def build_device_stats() -> dict:
    """Counters of this thread's last Cloud.build(device=True)."""
    c = (ctypes.c_int64 * 6)()
    ms = ctypes.c_double()
    check(_lib.lib().mknn_build_device_stats(c, ctypes.byref(ms)))
    return {"rounds": c[0], "tets": c[1], "conflicts": c[2], "tests": c[3], "deferred": c[4],
            "entries": c[5], "ms": ms.value}
