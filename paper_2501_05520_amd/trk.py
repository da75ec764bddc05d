"""Python binding of libtrk.so (ctypes).  Functions carry the C names and only
marshal arguments: torch device tensors become device pointers, the current HIP
stream is passed along, and status codes become exceptions.  Every step of the
tracking chain runs inside the library's HIP kernels; there is no Python or CPU
fallback, and loading fails loudly when the library is missing."""
import ctypes
import os
import struct

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# TRK_LIB names another build of the library (e.g. one compiled with other flags)
LIB_PATH = os.environ.get("TRK_LIB") or os.path.join(_PKG, "libtrk.so")

TRK_ABI_VERSION = 1
TRK_WEIGHTS_MAGIC = 0x5754524B
TRK_FP32, TRK_BF16, TRK_FP8, TRK_FP8_ALL, TRK_BF16_EMB32, TRK_BF16X3, TRK_BF16X3_GNN_BF16 = range(7)
STATUS = {0: "TRK_OK", -1: "TRK_E_INVAL", -2: "TRK_E_NOMEM", -3: "TRK_E_CAPACITY",
          -4: "TRK_E_DEVICE", -5: "TRK_E_WEIGHTS", -7: "TRK_E_EXPIRED", -8: "TRK_E_SHUTDOWN"}
EXPORTS = ("trk_create", "trk_destroy", "trk_embed", "trk_build_graph", "trk_build_graph_noalloc", "trk_filter",
           "trk_gnn", "trk_components", "trk_event", "trk_batch", "trk_strerror",
           "trk_server_create", "trk_server_submit", "trk_server_wait", "trk_server_stats",
           "trk_server_destroy", "trk_train_param_count", "trk_train_set_params", "trk_filter_train_fwd",
           "trk_filter_train_bwd", "trk_gnn_train_fwd", "trk_gnn_train_bwd", "trk_bce_with_logits",
           "trk_adam_update", "trk_embed_train_fwd", "trk_embed_train_bwd", "trk_pair_loss",
           "trk_service_start", "trk_service_stop", "trk_fit", "trk_probe_mfma", "trk_probe_copy")


class TrkError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


class trk_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32),
                ("emb_hidden", ctypes.c_int32), ("emb_layers", ctypes.c_int32), ("emb_dim", ctypes.c_int32),
                ("filt_hidden", ctypes.c_int32), ("filt_layers", ctypes.c_int32),
                ("gnn_hidden", ctypes.c_int32), ("gnn_iters", ctypes.c_int32),
                ("radius", ctypes.c_float), ("k_max", ctypes.c_int32),
                ("filter_cut", ctypes.c_float), ("score_cut", ctypes.c_float),
                ("precision", ctypes.c_int32),
                ("max_hits", ctypes.c_int64), ("max_cand_edges", ctypes.c_int64),
                ("max_kept_edges", ctypes.c_int64), ("max_events", ctypes.c_int32),
                ("stage_timing", ctypes.c_int32), ("training", ctypes.c_int32)]


class trk_event_info(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_int64), ("n_cand_edges", ctypes.c_int64),
                ("n_filt_edges", ctypes.c_int64), ("n_kept_edges", ctypes.c_int64),
                ("n_saturated", ctypes.c_int64), ("stage_ms", ctypes.c_float * 8)]

    STAGES = ("embed", "graph", "filter", "filter_cut", "gnn", "components")

    def as_dict(self):
        d = {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "stage_ms"}
        d["stage_ms"] = {name: float(self.stage_ms[i]) for i, name in enumerate(self.STAGES)}
        return d


class trk_server_config(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("max_batch_events", ctypes.c_int32),
                ("max_batch_hits", ctypes.c_int64), ("max_cand_edges", ctypes.c_int64),
                ("max_kept_edges", ctypes.c_int64), ("mem_budget_bytes", ctypes.c_uint64),
                ("bytes_per_hit", ctypes.c_uint64)]


class trk_server_info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "rejected", "expired", "batches",
                                              "batched_events", "admitted_at_once", "waited_for_memory")] + \
               [(k, ctypes.c_uint64) for k in ("inflight_bytes", "peak_inflight_bytes", "slot_bytes")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libtrk.so not found at {LIB_PATH}: build it with "
                               "`python -m paper_2501_05520_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, F, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_int32
        L.trk_create.argtypes = [ctypes.POINTER(trk_config), P, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(P)]
        L.trk_destroy.argtypes = [P]
        L.trk_destroy.restype = None
        L.trk_embed.argtypes = [P, P, I64, P, P]
        L.trk_build_graph.argtypes = [P, P, I64, P, P, I64, ctypes.POINTER(I64), ctypes.POINTER(I64), P]
        L.trk_build_graph_noalloc.argtypes = [P, I64, I32, F, I32, P, P, I64, ctypes.POINTER(I64),
                                              ctypes.POINTER(I64), P]
        L.trk_filter.argtypes = [P, P, I64, P, P, I64, P, P, P, I64, ctypes.POINTER(I64), P]
        L.trk_gnn.argtypes = [P, P, I64, P, P, I64, P, P]
        L.trk_components.argtypes = [P, I64, P, P, P, I64, F, P, P]
        L.trk_event.argtypes = [P, P, I64, P, ctypes.POINTER(trk_event_info), P]
        L.trk_batch.argtypes = [P, I32, P, P, P, ctypes.POINTER(trk_event_info), P]
        L.trk_server_create.argtypes = [ctypes.POINTER(trk_config), P, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.POINTER(trk_server_config), ctypes.POINTER(P)]
        L.trk_server_submit.argtypes = [P, P, I64, ctypes.c_double, ctypes.POINTER(I64)]
        L.trk_server_wait.argtypes = [P, I64, P, ctypes.POINTER(trk_event_info), ctypes.POINTER(ctypes.c_double)]
        L.trk_server_stats.argtypes = [P, ctypes.POINTER(trk_server_info)]
        L.trk_server_destroy.argtypes = [P]
        L.trk_server_destroy.restype = None
        L.trk_train_param_count.argtypes = [ctypes.POINTER(trk_config)]
        L.trk_train_set_params.argtypes = [P, P, P]
        L.trk_filter_train_fwd.argtypes = [P, P, I64, P, P, I64, P, P]
        L.trk_filter_train_bwd.argtypes = [P, P, I64, P, P, I64, P, P, P]
        L.trk_gnn_train_fwd.argtypes = [P, P, I64, P, P, I64, P, P]
        L.trk_gnn_train_bwd.argtypes = [P, P, I64, P, P, I64, P, P, P]
        L.trk_bce_with_logits.argtypes = [P, P, P, I64, P, ctypes.POINTER(F), P]
        L.trk_adam_update.argtypes = [P, P, P, P, P, I64, F, F, F, F, I64, P]
        L.trk_embed_train_fwd.argtypes = [P, P, I64, P, P]
        L.trk_embed_train_bwd.argtypes = [P, P, I64, P, P, P]
        L.trk_pair_loss.argtypes = [P, P, I64, P, P, P, I64, F, F, P, ctypes.POINTER(F), P]
        L.trk_fit.argtypes = [P, P, I64, P, I32, ctypes.c_double, P, P, P, I64, ctypes.POINTER(I64), P]
        L.trk_service_start.argtypes = [P, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(P),
                                        ctypes.POINTER(ctypes.c_int)]
        L.trk_service_stop.argtypes = [P]
        L.trk_service_stop.restype = None
        L.trk_strerror.argtypes = [ctypes.c_int]
        L.trk_strerror.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("trk_destroy", "trk_strerror", "trk_server_destroy", "trk_service_stop"):
                getattr(L, name).restype = ctypes.c_int
        L.trk_train_param_count.restype = ctypes.c_int64
        L.trk_probe_mfma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        L.trk_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise TrkError(rc, what)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# configuration and weights
# ---------------------------------------------------------------------------
def make_config(cfg, precision=TRK_FP32, max_hits=None, max_cand_edges=None, max_kept_edges=None, max_events=1,
                stage_timing=False, training=False):
    """trk_config from an object with the network and pipeline attributes
    (emb_hidden, emb_layers, emb_dim, filt_hidden, filt_layers, gnn_hidden,
    gnn_iters, radius, k_max, filter_cut, score_cut)."""
    if isinstance(precision, str):
        precision = {"fp32": TRK_FP32, "bf16": TRK_BF16, "fp8": TRK_FP8, "fp8all": TRK_FP8_ALL,
                     "bf16emb32": TRK_BF16_EMB32, "bf16x3": TRK_BF16X3,
                     "bf16x3gnn16": TRK_BF16X3_GNN_BF16}[precision]
    max_hits = int(max_hits)
    cand = int(max_cand_edges if max_cand_edges is not None else max_hits * cfg.k_max)
    kept = int(max_kept_edges if max_kept_edges is not None else cand)
    return trk_config(TRK_ABI_VERSION, cfg.emb_hidden, cfg.emb_layers, cfg.emb_dim, cfg.filt_hidden,
                      cfg.filt_layers, cfg.gnn_hidden, cfg.gnn_iters, float(cfg.radius), cfg.k_max,
                      float(cfg.filter_cut), float(cfg.score_cut), int(precision), max_hits, cand, kept,
                      int(max_events), int(bool(stage_timing)), int(bool(training)))


NET_ORDER = ("emb", "filt", "node_enc", "edge_enc", "edge_net", "node_net", "out")


def pack_weights(cfg, nets):
    """Weight blob of the C ABI: 16 uint32 header, then every layer's W[in][out]
    and b[out] as float32, networks in NET_ORDER."""
    hdr = [TRK_WEIGHTS_MAGIC, TRK_ABI_VERSION, cfg.emb_hidden, cfg.emb_layers, cfg.emb_dim, cfg.filt_hidden,
           cfg.filt_layers, cfg.gnn_hidden, cfg.gnn_iters] + [0] * 7
    parts = [struct.pack("<16I", *hdr)]
    for name in NET_ORDER:
        for w, b in nets[name]:
            parts.append(np.ascontiguousarray(w, dtype=np.float32).tobytes())
            parts.append(np.ascontiguousarray(b, dtype=np.float32).tobytes())
    return b"".join(parts)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def trk_create(config, weights_blob, device=0):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(weights_blob, len(weights_blob))
    _check(lib().trk_create(ctypes.byref(config), buf, len(weights_blob), int(device), ctypes.byref(h)),
           "trk_create")
    return h


def trk_destroy(ctx):
    lib().trk_destroy(ctx)


def trk_embed(ctx, x, emb, stream=None):
    _check(lib().trk_embed(ctx, _ptr(x), x.shape[0], _ptr(emb), _stream(stream)), "trk_embed")


def trk_build_graph(ctx, emb, src, dst, stream=None, truncate_ok=False):
    """Returns (total edge count, saturated count).  With truncate_ok a total above
    the capacity is returned instead of raised: the first src.numel() edges of the
    sorted list are then written."""
    ne, ns = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().trk_build_graph(ctx, _ptr(emb), emb.shape[0], _ptr(src), _ptr(dst), src.numel(),
                               ctypes.byref(ne), ctypes.byref(ns), _stream(stream))
    if rc == -3 and truncate_ok:
        return ne.value, ns.value
    if rc == -3:
        raise TrkError(rc, f"trk_build_graph (needs {ne.value} edges)")
    _check(rc, "trk_build_graph")
    return ne.value, ns.value


def trk_build_graph_noalloc(emb, radius, k_max, src, dst, stream=None):
    """Context-free, allocation-free radius graph on the current device; returns
    (total edge count, saturated count)."""
    ne, ns = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().trk_build_graph_noalloc(_ptr(emb), emb.shape[0], emb.shape[1] if emb.dim() == 2 else 0,
                                       float(radius), int(k_max), _ptr(src), _ptr(dst), src.numel(),
                                       ctypes.byref(ne), ctypes.byref(ns), _stream(stream))
    if rc == -3:
        raise TrkError(rc, f"trk_build_graph_noalloc (needs {ne.value} edges)")
    _check(rc, "trk_build_graph_noalloc")
    return ne.value, ns.value


def trk_filter(ctx, emb, src, dst, scores, kept_src, kept_dst, stream=None):
    nk = ctypes.c_int64()
    rc = lib().trk_filter(ctx, _ptr(emb), emb.shape[0], _ptr(src), _ptr(dst), src.numel(), _ptr(scores),
                          _ptr(kept_src), _ptr(kept_dst), kept_src.numel(), ctypes.byref(nk), _stream(stream))
    if rc == -3:
        raise TrkError(rc, f"trk_filter (needs {nk.value} kept edges)")
    _check(rc, "trk_filter")
    return nk.value


def trk_gnn(ctx, x, src, dst, scores, stream=None):
    _check(lib().trk_gnn(ctx, _ptr(x), x.shape[0], _ptr(src), _ptr(dst), src.numel(), _ptr(scores),
                         _stream(stream)), "trk_gnn")


def trk_components(ctx, n, src, dst, scores, cut, labels, stream=None):
    _check(lib().trk_components(ctx, int(n), _ptr(src), _ptr(dst), _ptr(scores), src.numel(), float(cut),
                                _ptr(labels), _stream(stream)), "trk_components")


def trk_event(ctx, x, labels, stream=None):
    info = trk_event_info()
    _check(lib().trk_event(ctx, _ptr(x), x.shape[0], _ptr(labels), ctypes.byref(info), _stream(stream)),
           "trk_event")
    return info.as_dict()


def trk_batch(ctx, x, offsets, labels, stream=None):
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    nev = offs.size - 1
    infos = (trk_event_info * max(nev, 1))()
    _check(lib().trk_batch(ctx, nev, _ptr(x), offs.ctypes.data_as(ctypes.c_void_p), _ptr(labels), infos,
                           _stream(stream)), "trk_batch")
    return [infos[i].as_dict() for i in range(nev)]


def trk_strerror(status):
    return lib().trk_strerror(int(status)).decode()


# ---------------------------------------------------------------------------
# convenience wrapper owning a context and its output buffers
# ---------------------------------------------------------------------------
class Pipeline:
    """A context plus allocation of outputs; each method returns torch tensors."""

    def __init__(self, cfg, nets, precision="fp32", device=0, max_hits=None, max_cand_edges=None,
                 max_kept_edges=None, max_events=1, stage_timing=False):
        self.cfg = cfg
        self.device = torch.device("cuda", device)
        self.config = make_config(cfg, precision, max_hits, max_cand_edges, max_kept_edges, max_events,
                                  stage_timing)
        self.ctx = trk_create(self.config, pack_weights(cfg, nets), device)

    def close(self):
        if self.ctx is not None:
            trk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, a):
        if not torch.is_tensor(a):
            a = torch.as_tensor(np.asarray(a, dtype=np.float32))
        return a.to(device=self.device, dtype=torch.float32).contiguous()

    def _i32(self, a):
        if not torch.is_tensor(a):
            a = torch.as_tensor(np.asarray(a, dtype=np.int64))
        return a.to(device=self.device, dtype=torch.int32).contiguous()

    def embed(self, x):
        x = self._f32(x)
        emb = torch.empty((x.shape[0], self.cfg.emb_dim), dtype=torch.float32, device=self.device)
        trk_embed(self.ctx, x, emb)
        return emb

    def build_graph(self, emb, cap=None):
        emb = self._f32(emb)
        cap = int(cap if cap is not None else self.config.max_cand_edges)
        src = torch.empty(cap, dtype=torch.int32, device=self.device)
        dst = torch.empty(cap, dtype=torch.int32, device=self.device)
        ne, ns = trk_build_graph(self.ctx, emb, src, dst)
        return src[:ne], dst[:ne], ns

    def filter(self, emb, src, dst, cap=None):
        emb, src, dst = self._f32(emb), self._i32(src), self._i32(dst)
        m = src.numel()
        cap = int(cap if cap is not None else m)
        scores = torch.empty(m, dtype=torch.float32, device=self.device)
        ks = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)[:cap]
        kd = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)[:cap]
        nk = trk_filter(self.ctx, emb, src, dst, scores, ks, kd)
        return scores, ks[:nk], kd[:nk]

    def gnn(self, x, src, dst):
        x, src, dst = self._f32(x), self._i32(src), self._i32(dst)
        scores = torch.empty(src.numel(), dtype=torch.float32, device=self.device)
        trk_gnn(self.ctx, x, src, dst, scores)
        return scores

    def components(self, n, src, dst, scores=None, cut=0.5):
        src, dst = self._i32(src), self._i32(dst)
        scores = None if scores is None else self._f32(scores)
        labels = torch.empty(max(int(n), 1), dtype=torch.int32, device=self.device)[:int(n)]
        trk_components(self.ctx, n, src, dst, scores, cut, labels)
        return labels

    def event(self, x):
        x = self._f32(x)
        labels = torch.empty(max(x.shape[0], 1), dtype=torch.int32, device=self.device)[:x.shape[0]]
        info = trk_event(self.ctx, x, labels)
        return labels, info

    def batch(self, x, offsets):
        x = self._f32(x)
        labels = torch.empty(max(x.shape[0], 1), dtype=torch.int32, device=self.device)[:x.shape[0]]
        infos = trk_batch(self.ctx, x, offsets, labels)
        return labels, infos


# ---------------------------------------------------------------------------
# serving loop
# ---------------------------------------------------------------------------
def trk_server_create(config, weights_blob, device, server_config):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(weights_blob, len(weights_blob))
    _check(lib().trk_server_create(ctypes.byref(config), buf, len(weights_blob), int(device),
                                   ctypes.byref(server_config), ctypes.byref(h)), "trk_server_create")
    return h


def trk_server_submit(srv, x, deadline_ms=0.0):
    """x: host float32 [n, 3]; returns the ticket."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = ctypes.c_int64()
    _check(lib().trk_server_submit(srv, x.ctypes.data_as(ctypes.c_void_p), x.shape[0], float(deadline_ms),
                                   ctypes.byref(t)), "trk_server_submit")
    return t.value


def trk_server_wait(srv, ticket, n):
    """Returns (status, labels int32 [n], info dict, latency ms)."""
    labels = np.empty(max(int(n), 1), dtype=np.int32)
    info = trk_event_info()
    lat = ctypes.c_double()
    rc = lib().trk_server_wait(srv, int(ticket), labels.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info),
                               ctypes.byref(lat))
    return rc, labels[:int(n)], info.as_dict(), lat.value


def trk_server_stats(srv):
    st = trk_server_info()
    _check(lib().trk_server_stats(srv, ctypes.byref(st)), "trk_server_stats")
    return st.as_dict()


def trk_server_destroy(srv):
    lib().trk_server_destroy(srv)


def trk_fit(ctx, x, labels, min_hits=3, b_field=2.0, cap=None, stream=None):
    """Helix fit of the candidates of labels[n] over x[n][3] (device tensors);
    returns (labels int32 [c], n_hits int32 [c], params float64 [c][6])."""
    n = x.shape[0]
    cap = int(cap if cap is not None else max(n // 3, 1))
    dev = x.device
    cl = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    cn = torch.empty_like(cl)
    par = torch.empty((max(cap, 1), 6), dtype=torch.float64, device=dev)
    nc = ctypes.c_int64()
    rc = lib().trk_fit(ctx, _ptr(x), n, _ptr(labels), int(min_hits), float(b_field), _ptr(cl), _ptr(cn), _ptr(par),
                       cap, ctypes.byref(nc), _stream(stream))
    if rc != 0:
        raise TrkError(rc, f"trk_fit (needs {nc.value} candidates)")
    k = nc.value
    return cl[:k], cn[:k], par[:k]


def trk_service_start(srv, host="127.0.0.1", port=0):
    """Starts the TCP front end of a server; returns (handle, bound port)."""
    h = ctypes.c_void_p()
    bound = ctypes.c_int()
    _check(lib().trk_service_start(srv, host.encode() if host else None, int(port), ctypes.byref(h),
                                   ctypes.byref(bound)), "trk_service_start")
    return h, bound.value


def trk_service_stop(svc):
    lib().trk_service_stop(svc)


SERVICE_REQ_MAGIC, SERVICE_RESP_MAGIC = 0x5154524B, 0x5254524B


class ServiceClient:
    """A blocking client of the TCP front end (wire format in include/trk.h); one
    connection, requests in order.  Pure host code: usable without a GPU."""

    _REQ = struct.Struct("<IIqd")
    _RESP = struct.Struct("<Iiqd5q8f")

    def __init__(self, host, port, timeout=60.0):
        import socket
        self.sock = socket.create_connection((host, int(port)), timeout=timeout)
        self.sock.setsockopt(socket.IPPROTO_TCP, socket.TCP_NODELAY, 1)

    def _recv(self, n):
        buf = bytearray(n)
        view, got = memoryview(buf), 0
        while got < n:
            k = self.sock.recv_into(view[got:], n - got)
            if k == 0:
                raise ConnectionError("service closed the connection")
            got += k
        return bytes(buf)

    def request(self, x, deadline_ms=0.0):
        """Returns (status, labels int32 [n] or None, info dict, server latency ms)."""
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
        n = x.shape[0]
        self.sock.sendall(self._REQ.pack(SERVICE_REQ_MAGIC, 0, n, float(deadline_ms)) + x.tobytes())
        magic, status, rn, lat, *rest = self._RESP.unpack(self._recv(self._RESP.size))
        if magic != SERVICE_RESP_MAGIC or rn != n:
            raise ConnectionError("malformed response")
        counts, stage = rest[:5], rest[5:]
        info = dict(zip(("n_hits", "n_cand_edges", "n_filt_edges", "n_kept_edges", "n_saturated"), counts))
        info["stage_ms"] = dict(zip(trk_event_info.STAGES, stage))
        labels = np.frombuffer(self._recv(4 * n), dtype=np.int32) if status == 0 and n > 0 else \
            (np.zeros(0, np.int32) if status == 0 else None)
        return status, labels, info, lat

    def close(self):
        self.sock.close()


class Server:
    """A serving loop on one GPU; submit/wait may be called from many threads."""

    def __init__(self, cfg, nets, precision="bf16", device=0, n_slots=2, max_batch_events=8,
                 max_batch_hits=220000, mem_budget_bytes=64 << 30, max_cand_edges=0, max_kept_edges=0,
                 bytes_per_hit=0, stage_timing=False):
        self.cfg = cfg
        config = make_config(cfg, precision, max_batch_hits, max_cand_edges or None, max_kept_edges or None,
                             max_batch_events, stage_timing)
        scfg = trk_server_config(int(n_slots), int(max_batch_events), int(max_batch_hits), int(max_cand_edges),
                                 int(max_kept_edges), int(mem_budget_bytes), int(bytes_per_hit))
        self.h = trk_server_create(config, pack_weights(cfg, nets), device, scfg)

    def submit(self, x, deadline_ms=0.0):
        return trk_server_submit(self.h, x, deadline_ms)

    def wait(self, ticket, n):
        return trk_server_wait(self.h, ticket, n)

    def stats(self):
        return trk_server_stats(self.h)

    def close(self):
        if self.h is not None:
            trk_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# training entry points
# ---------------------------------------------------------------------------
TRAIN_NETS = ("filt", "node_enc", "edge_enc", "edge_net", "node_net", "out", "emb")


def trk_train_param_count(config):
    return int(lib().trk_train_param_count(ctypes.byref(config)))


def flatten_params(nets):
    """Flat FP32 parameter vector of the trained networks (C-ABI layout)."""
    parts = []
    for name in TRAIN_NETS:
        for w, b in nets[name]:
            parts += [np.ascontiguousarray(w, np.float32).reshape(-1), np.ascontiguousarray(b, np.float32)]
    return np.concatenate(parts)


def unflatten_params(vec, nets_like):
    """Inverse of flatten_params, shaped like nets_like (numpy)."""
    vec = np.asarray(vec)
    out, o = {}, 0
    for name in TRAIN_NETS:
        layers = []
        for w, b in nets_like[name]:
            W = vec[o:o + w.size].reshape(w.shape); o += w.size
            B = vec[o:o + b.size]; o += b.size
            layers.append((W, B))
        out[name] = layers
    assert o == vec.size
    return out


def trk_train_set_params(ctx, params, stream=None):
    _check(lib().trk_train_set_params(ctx, _ptr(params), _stream(stream)), "trk_train_set_params")


def trk_filter_train_fwd(ctx, emb, src, dst, logits, stream=None):
    _check(lib().trk_filter_train_fwd(ctx, _ptr(emb), emb.shape[0], _ptr(src), _ptr(dst), src.numel(), _ptr(logits),
                                      _stream(stream)), "trk_filter_train_fwd")


def trk_filter_train_bwd(ctx, emb, src, dst, dlogits, grads, stream=None):
    _check(lib().trk_filter_train_bwd(ctx, _ptr(emb), emb.shape[0], _ptr(src), _ptr(dst), src.numel(),
                                      _ptr(dlogits), _ptr(grads), _stream(stream)), "trk_filter_train_bwd")


def trk_gnn_train_fwd(ctx, x, src, dst, logits, stream=None):
    _check(lib().trk_gnn_train_fwd(ctx, _ptr(x), x.shape[0], _ptr(src), _ptr(dst), src.numel(), _ptr(logits),
                                   _stream(stream)), "trk_gnn_train_fwd")


def trk_gnn_train_bwd(ctx, x, src, dst, dlogits, grads, stream=None):
    _check(lib().trk_gnn_train_bwd(ctx, _ptr(x), x.shape[0], _ptr(src), _ptr(dst), src.numel(), _ptr(dlogits),
                                   _ptr(grads), _stream(stream)), "trk_gnn_train_bwd")


def trk_bce_with_logits(ctx, logits, targets, dlogits, stream=None):
    loss = ctypes.c_float()
    _check(lib().trk_bce_with_logits(ctx, _ptr(logits), _ptr(targets), logits.numel(), _ptr(dlogits),
                                     ctypes.byref(loss), _stream(stream)), "trk_bce_with_logits")
    return loss.value


def trk_adam_update(ctx, params, grads, m, v, lr, beta1, beta2, eps, step, stream=None):
    _check(lib().trk_adam_update(ctx, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(), float(lr),
                                 float(beta1), float(beta2), float(eps), int(step), _stream(stream)),
           "trk_adam_update")


def trk_embed_train_fwd(ctx, x, emb, stream=None):
    _check(lib().trk_embed_train_fwd(ctx, _ptr(x), x.shape[0], _ptr(emb), _stream(stream)), "trk_embed_train_fwd")


def trk_embed_train_bwd(ctx, x, demb, grads, stream=None):
    _check(lib().trk_embed_train_bwd(ctx, _ptr(x), x.shape[0], _ptr(demb), _ptr(grads), _stream(stream)),
           "trk_embed_train_bwd")


def trk_pair_loss(ctx, emb, pa, pb, y, margin, demb, neg_weight=1.0, stream=None):
    loss = ctypes.c_float()
    _check(lib().trk_pair_loss(ctx, _ptr(emb), emb.shape[0], _ptr(pa), _ptr(pb), _ptr(y), pa.numel(), float(margin),
                               float(neg_weight), _ptr(demb), ctypes.byref(loss), _stream(stream)), "trk_pair_loss")
    return loss.value


# ---------------------------------------------------------------------------
# roofline denominators measured on the device
# ---------------------------------------------------------------------------
def trk_probe_mfma(precision, iters, device=0):
    """Dense MFMA rate (TFLOP/s) of 'fp32', 'bf16' or 'fp8' measured on `device`."""
    prec = {"fp32": TRK_FP32, "bf16": TRK_BF16, "fp8": TRK_FP8}[precision]
    out = ctypes.c_double()
    _check(lib().trk_probe_mfma(int(device), prec, int(iters), ctypes.byref(out)), "trk_probe_mfma")
    return out.value


def trk_probe_copy(src, dst, reps=5, stream=None):
    """HBM GB/s (read + write) of a device-to-device copy of src into dst (same byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    out = ctypes.c_double()
    _check(lib().trk_probe_copy(_ptr(src), _ptr(dst), nbytes, int(reps), _stream(stream), ctypes.byref(out)),
           "trk_probe_copy")
    return out.value
