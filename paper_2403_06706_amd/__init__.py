"""MI355X guiding-centre electron pusher: Python binding of libgcpush.so.

Argument marshalling only.  Every step of the method runs in the HIP kernels
behind the C ABI (include/gcpush.h); torch supplies device buffers for
outputs and the HIP stream.  Importing this package needs the built library
(it raises ImportError otherwise); using a context needs a GPU.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from typing import Dict, Optional

import numpy as np

from . import _abi
from ._abi import (GC_F64, GC_F32, GC_F16, GC_PREC_F64, GC_PREC_F32_ACC64, GC_PREC_F32_KAHAN,  # noqa: F401
                   GC_ACTIVE, GC_EXITED, GC_FINISHED, GC_NONFINITE, GC_FLAG_BOOTSTRAP, GC_FLAG_PENDING,
                   GC_ORDER_NONE, GC_ORDER_COMPACT, GC_ORDER_BIN, GC_SOURCE_GRID, GC_SOURCE_MLP,
                   GC_MLP_PARAMS, STATE_DOUBLES, STATE_U32)

lib = _abi.load()

_DTYPES = {"f64": GC_F64, "f32": GC_F32, "f16": GC_F16}
_PRECS = {"f64": GC_PREC_F64, "f32_acc64": GC_PREC_F32_ACC64, "f32_kahan": GC_PREC_F32_KAHAN}
_ORDERS = {"none": GC_ORDER_NONE, "compact": GC_ORDER_COMPACT, "bin": GC_ORDER_BIN}
_SOURCES = {"grid": GC_SOURCE_GRID, "mlp": GC_SOURCE_MLP}
MLP_DEPTH, MLP_WIDTH, MLP_OUT = 6, 128, 6


def mlp_flatten(params: Dict[str, np.ndarray]) -> np.ndarray:
    """{W1..W6 [128,128], c1..c6 [128], Wo [6,128], co [6]} -> the GC_MLP_PARAMS float32 block."""
    parts = [np.asarray(params[f"W{l}"]).ravel() for l in range(1, MLP_DEPTH + 1)]
    parts += [np.asarray(params[f"c{l}"]).ravel() for l in range(1, MLP_DEPTH + 1)]
    parts += [np.asarray(params["Wo"]).ravel(), np.asarray(params["co"]).ravel()]
    flat = np.concatenate(parts).astype(np.float32)
    if flat.size != GC_MLP_PARAMS:
        raise ValueError(f"expected {GC_MLP_PARAMS} parameters, got {flat.size}")
    return flat


def mlp_unflatten(flat: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for l in range(1, MLP_DEPTH + 1):
        out[f"W{l}"] = flat[o:o + MLP_WIDTH * MLP_WIDTH].reshape(MLP_WIDTH, MLP_WIDTH)
        o += MLP_WIDTH * MLP_WIDTH
    for l in range(1, MLP_DEPTH + 1):
        out[f"c{l}"] = flat[o:o + MLP_WIDTH]
        o += MLP_WIDTH
    out["Wo"] = flat[o:o + MLP_OUT * MLP_WIDTH].reshape(MLP_OUT, MLP_WIDTH)
    o += MLP_OUT * MLP_WIDTH
    out["co"] = flat[o:o + MLP_OUT]
    return out


# Contexts still open at interpreter exit are closed while torch is alive
# (their memory may come from torch's allocator through callbacks).
_live = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for ctx in list(_live):
        ctx.close()


class GCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gc status {status}: {message}")
        self.status = status


def _torch():
    import torch
    return torch


class Context:
    """One gc_ctx on one device, using torch's current stream unless one is given."""

    def __init__(self, device: int = 0, precision: str = "f64", order: str = "bin", chunk_steps: int = 64,
                 bin_coarsen: int = 0, block_size: Optional[int] = None, persistent: bool = False, tile: int = 1024,
                 log_depth: int = 0, timing=False, field_source: str = "grid", tail_threshold: Optional[int] = None,
                 stream=None, allocator: str = "torch"):
        """allocator "torch" (default): the context's device memory comes from
        torch's caching allocator, on the context's stream; "hip": from hipMalloc.
        timing: False/0 off, True/1 events on pushes and reorders, 2 or "push"
        on pushes only (gc_options.timing)."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the guiding-centre pusher runs only on the device")
        self.device = device
        self._stream = stream if stream is not None else torch.cuda.current_stream(device)
        o = _abi.gc_options()
        lib.gc_default_options(C.byref(o))
        o.hip_stream = self._stream.cuda_stream
        o.device = device
        o.precision = _PRECS[precision]
        o.order = _ORDERS[order]
        o.chunk_steps = chunk_steps
        o.bin_coarsen = bin_coarsen
        if block_size is not None:          # else the library's default
            o.block_size = block_size
        o.persistent = int(persistent)
        o.tile = tile
        o.log_depth = log_depth
        o.timing = 2 if timing == "push" else int(timing)
        o.field_source = _SOURCES[field_source]
        if tail_threshold is not None:
            o.tail_threshold = int(tail_threshold)
        self._alloc_fns = None
        if allocator == "torch":
            stream_ = self._stream

            def _alloc(nbytes, _user):
                try:
                    return torch.cuda.caching_allocator_alloc(max(int(nbytes), 1), device=device, stream=stream_)
                except RuntimeError:
                    return None

            def _free(ptr, _user):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc_fns = (_abi.DEV_ALLOC_FN(_alloc), _abi.DEV_FREE_FN(_free))
            o.dev_alloc, o.dev_free = self._alloc_fns
        elif allocator != "hip":
            raise ValueError(f"unknown allocator {allocator!r}")
        self._opt = o
        h = C.c_void_p()
        st = lib.gc_create(C.byref(h), C.byref(o))
        self._h = h
        if st != 0:
            msg = lib.gc_last_error(h).decode() if h else ""
            if h:
                lib.gc_destroy(h)
            self._h = None
            raise GCError(st, msg)
        self.log_depth = log_depth
        _live.add(self)

    # -------------------------------------------------------------- basics
    def _check(self, st: int):
        if st != 0:
            raise GCError(st, lib.gc_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.gc_destroy(self._h)     # may call the allocator callbacks, kept alive until here
            self._h = None
        self._alloc_fns = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    @property
    def stream(self):
        return self._stream

    # Library work runs on the context's stream; torch work on the caller's
    # current stream.  Order them explicitly around buffers that cross (on one
    # stream the order is already the issue order, and a wait would only add a
    # marker packet to the queue).
    def _inputs_ready(self):
        cur = _torch().cuda.current_stream(self.device)
        if cur != self._stream:
            self._stream.wait_stream(cur)

    def _outputs_ready(self, *tensors):
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur == self._stream:
            return
        for t in tensors:
            t.record_stream(self._stream)
        cur.wait_stream(self._stream)

    def set_options(self, **kw):
        o = _abi.gc_options()
        self._check(lib.gc_get_options(self._h, C.byref(o)))
        for k, v in kw.items():
            if k == "precision" and isinstance(v, str):
                v = _PRECS[v]
            elif k == "order" and isinstance(v, str):
                v = _ORDERS[v]
            elif k == "field_source" and isinstance(v, str):
                v = _SOURCES[v]
            elif k == "stream":
                self._stream = v
                k, v = "hip_stream", v.cuda_stream
            setattr(o, k, int(v) if not isinstance(v, int) and k != "hip_stream" else v)
        self._check(lib.gc_set_options(self._h, C.byref(o)))

    def count(self) -> int:
        n = C.c_uint64()
        self._check(lib.gc_count(self._h, C.byref(n)))
        return n.value

    # --------------------------------------------------------------- field
    def load_field(self, grid, data: np.ndarray, store_dtype: str = "f64", extra: Optional[np.ndarray] = None):
        """data [nr][nth][nph][12]; extra (optional, same dtype) [nr][nth][nph][9]:
        the node values that switch the push to the full Eqs. 1-2."""
        arr = np.ascontiguousarray(data)
        if arr.dtype not in (np.float64, np.float32):
            raise TypeError("field data must be float64 or float32")
        if arr.size != grid.nr * grid.nth * grid.nph * 12:
            raise ValueError(f"field data must hold [nr][nth][nph][12] = {grid.nr * grid.nth * grid.nph * 12} values "
                             f"(got {arr.size})")
        xp = None
        if extra is not None:
            xarr = np.ascontiguousarray(extra, dtype=arr.dtype)
            if xarr.shape != (grid.nr, grid.nth, grid.nph, 9):
                raise ValueError("extra must be [nr][nth][nph][9]")
            xp = xarr.ctypes.data
        d = _abi.gc_field_desc(grid.nr, grid.nth, grid.nph, GC_F64 if arr.dtype == np.float64 else GC_F32,
                               grid.r_min, grid.r_max, arr.ctypes.data, _DTYPES[store_dtype], 0, xp)
        self._check(lib.gc_load_field(self._h, C.byref(d)))

    # ----------------------------------------------------------- injection
    def inject(self, ens, first_id: int = 0, n: Optional[int] = None):
        """ens: object with the attributes of synthetic.workloads.Ensemble."""
        d = _abi.gc_inject_desc(ens.ensemble, first_id, ens.n if n is None else n, ens.seed, ens.q, ens.m, ens.ekin,
                                ens.r0, ens.lat0, ens.lon0, ens.dlon, ens.dr0, ens.dlat, ens.mu_lo, ens.mu_hi,
                                ens.lambda_par, ens.r_in, ens.r_out, int(ens.max_steps), int(ens.drift_free),
                                int(ens.scatter_law), int(getattr(ens, "rebirth_steps", 0)),
                                float(getattr(ens, "v_wind", 0.0)))
        self._check(lib.gc_inject(self._h, C.byref(d)))

    # ------------------------------------------------------------- advance
    def advance(self, dt: float, n_steps: int):
        self._check(lib.gc_advance(self._h, float(dt), int(n_steps)))

    def advance_graph(self, dt: float, n_steps: int):
        self._check(lib.gc_advance_graph(self._h, float(dt), int(n_steps)))

    # ------------------------------------------------------------- moments
    @staticmethod
    def _spec(spec, accumulate: bool = False) -> _abi.gc_moment_spec:
        return _abi.gc_moment_spec(spec.n_rbins, spec.r_lo, spec.r_hi, spec.n_mubins, spec.sel_r_lo, spec.sel_r_hi,
                                   spec.age_lo, spec.age_hi, spec.min_collisions, spec.n_agebins, spec.age_max,
                                   spec.n_ebins, spec.e_lo, spec.e_hi, spec.e_unit, spec.len_unit,
                                   int(getattr(spec, "min_birth", 0)), 1 if accumulate else 0)

    def moments_size(self, spec) -> int:
        return int(lib.gc_moments_size(C.byref(self._spec(spec))))

    def moments(self, spec, out=None, accumulate: bool = False):
        """Snapshot statistics into a new int64 device tensor, or into out (a
        contiguous int64 device tensor of at least the moments size), replacing
        its contents or, with accumulate, adding to them on the device (the sum
        over snapshots).  Returns the moments view of the output."""
        torch = _torch()
        if accumulate and out is None:
            raise ValueError("accumulate needs out")
        s = self._spec(spec, accumulate=accumulate)
        m = int(lib.gc_moments_size(C.byref(s)))
        if out is None:
            out = torch.empty(max(m, 1), dtype=torch.int64, device=f"cuda:{self.device}")
        elif out.dtype != torch.int64 or out.numel() < m or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous int64 tensor of at least {m} values")
        self._inputs_ready()
        self._check(lib.gc_moments(self._h, C.byref(s), C.c_void_p(out.data_ptr())))
        self._outputs_ready(out)
        return out[:m]

    # --------------------------------------------------------------- state
    def get_state(self) -> Dict[str, "object"]:
        torch = _torch()
        n = self.count()
        dev = f"cuda:{self.device}"
        out = {k: torch.empty(max(n, 1), dtype=torch.float64, device=dev) for k in STATE_DOUBLES}
        out.update({k: torch.empty(max(n, 1), dtype=torch.int32, device=dev) for k in STATE_U32})
        v = _abi.gc_state_view(**{k: t.data_ptr() for k, t in out.items()})
        self._inputs_ready()
        self._check(lib.gc_get_state(self._h, C.byref(v)))
        self._outputs_ready(*out.values())
        return {k: t[:n] for k, t in out.items()}

    def set_state(self, state: Dict[str, "object"]):
        torch = _torch()
        n = int(state["r"].shape[0])
        keep = {}
        for k in STATE_DOUBLES:
            keep[k] = state[k].to(device=f"cuda:{self.device}", dtype=torch.float64).contiguous()
        for k in STATE_U32:
            keep[k] = state[k].to(device=f"cuda:{self.device}", dtype=torch.int32).contiguous()
        v = _abi.gc_state_view(**{k: t.data_ptr() for k, t in keep.items()})
        self._inputs_ready()
        self._check(lib.gc_set_state(self._h, C.byref(v), n))
        self._stream.synchronize()   # the buffers above may be freed on return

    def get_log(self):
        torch = _torch()
        n = self.count()
        out = torch.empty((max(n, 1), max(self.log_depth, 1)), dtype=torch.int32, device=f"cuda:{self.device}")
        self._inputs_ready()
        self._check(lib.gc_get_log(self._h, C.c_void_p(out.data_ptr())))
        self._outputs_ready(out)
        return out[:n]

    def get_order(self, keys: bool = True):
        """Slot order after the last reorder (gc_get_order): (slot -> global
        index, slot -> sorted cell key or None, live count at that reorder),
        as device int32 tensors and an int."""
        torch = _torch()
        n = self.count()
        dev = f"cuda:{self.device}"
        gid = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        key = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if keys else None
        live = torch.empty(1, dtype=torch.int32, device=dev)
        self._inputs_ready()
        self._check(lib.gc_get_order(self._h, C.c_void_p(gid.data_ptr()),
                                     C.c_void_p(key.data_ptr()) if keys else None, C.c_void_p(live.data_ptr())))
        self._outputs_ready(gid, live, *([key] if keys else []))
        return gid[:n], (key[:n] if keys else None), int(live.item())

    # ------------------------------------------------------------ counters
    def counters(self) -> dict:
        c = _abi.gc_counters()
        self._check(lib.gc_get_counters(self._h, C.byref(c)))
        return {"push_ms": c.push_ms, "n_push": c.n_push, "reorder_ms": c.reorder_ms, "n_reorder": c.n_reorder,
                "particle_steps": c.particle_steps, "form_ms": list(c.form_ms),
                "form_launches": list(c.form_launches), "form_steps": list(c.form_steps)}

    def reset_counters(self):
        self._check(lib.gc_reset_counters(self._h))

    def options(self) -> dict:
        o = _abi.gc_options()
        self._check(lib.gc_get_options(self._h, C.byref(o)))
        return {"precision": o.precision, "order": o.order, "chunk_steps": o.chunk_steps,
                "bin_coarsen": o.bin_coarsen, "block_size": o.block_size, "persistent": o.persistent,
                "tile": o.tile, "field_source": o.field_source, "tail_threshold": o.tail_threshold}

    def autotune(self, dt: float, probe_steps: int = 128, blocks=(64, 128, 256), coarsen=(0, 1, 2),
                 chunks=(), tiles=(256, 1024, 4096), cache: Optional[str] = None, key: Optional[str] = None) -> dict:
        """Time candidate launch parameters on this context's particles (see
        gc_autotune) and apply the best.  With cache and key, a stored choice is
        applied without timing, and a new choice is stored."""
        import json
        import os
        if cache and key and os.path.exists(cache):
            with open(cache) as f:
                stored_all = json.load(f)
            if key in stored_all:
                chosen = stored_all[key]
                self.set_options(**{k: v for k, v in chosen["options"].items() if k != "precision"})
                return dict(chosen, cached=True)
        sp = _abi.gc_tune_space()
        for name, vals, cap in (("block", blocks, 3), ("coarsen", coarsen, 4), ("chunk", chunks, 6), ("tile", tiles, 4)):
            vals = list(vals)[:cap]
            setattr(sp, "n_" + name, len(vals))
            arr = getattr(sp, name)
            for i, v in enumerate(vals):
                arr[i] = int(v)
        sp.probe_steps = int(probe_steps)
        sp.dt = float(dt)
        res = _abi.gc_tune_result()
        self._check(lib.gc_autotune(self._h, C.byref(sp), C.byref(res)))
        out = {"options": self.options(), "best_rate": res.best_rate, "default_rate": res.default_rate,
               "n_tried": res.n_tried, "cached": False}
        if cache and key:
            stored_all = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    stored_all = json.load(f)
            stored_all[key] = {k: out[k] for k in ("options", "best_rate", "default_rate", "n_tried")}
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(stored_all, f, indent=1)
        return out

    # -------------------------------------------------------- neural field
    def mlp_set(self, freq, r_ref: float, scale, power, params: Optional[Dict[str, np.ndarray]] = None):
        """Install the network (gc_mlp_set).  freq [64, 3] (a_j, b_j, n_j)."""
        d = _abi.gc_mlp_desc()
        fq = np.asarray(freq, dtype=np.float64)
        for j in range(64):
            for i in range(3):
                d.freq[j][i] = float(fq[j, i])
        d.r_ref = float(r_ref)
        for c in range(6):
            d.scale[c] = float(scale[c])
            d.power[c] = float(power[c])
        keep = None
        if params is not None:
            keep = mlp_flatten(params)
            d.params = keep.ctypes.data_as(C.POINTER(C.c_float))
        self._inputs_ready()
        self._check(lib.gc_mlp_set(self._h, C.byref(d)))

    def _mlp_block(self, fn) -> Dict[str, np.ndarray]:
        flat = np.empty(GC_MLP_PARAMS, dtype=np.float32)
        self._check(fn(self._h, flat.ctypes.data_as(C.POINTER(C.c_float))))
        return mlp_unflatten(flat)

    def mlp_params(self) -> Dict[str, np.ndarray]:
        return self._mlp_block(lib.gc_mlp_get_params)

    def mlp_grads(self) -> Dict[str, np.ndarray]:
        return self._mlp_block(lib.gc_mlp_get_grads)

    def mlp_train_step(self, pts, tgt, wc=(1.0,) * 6, beta_pair: float = 0.0, lr: float = 1e-3,
                       betas=(0.9, 0.999), eps: float = 1e-8, step: int = 1, apply: bool = True,
                       noalloc: bool = False) -> float:
        """One training step (gc_mlp_train_step, or with noalloc the variant with
        the library's static workspace, gc_mlp_train_step_noalloc).  pts: device
        float64 [3, 2n] (point n + i pairs with point i); tgt: device float64 [2n, 6]."""
        n2 = int(pts.shape[1])
        if pts.shape[0] != 3 or n2 % 2 or tuple(tgt.shape) != (n2, 6):
            raise ValueError("pts must be [3, 2n] and tgt [2n, 6]")
        for t in (pts, tgt):
            if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float64"):
                raise TypeError("pts and tgt must be contiguous float64 device tensors")
        o = _abi.gc_mlp_train_opts()
        o.lr, o.beta1, o.beta2, o.eps = float(lr), float(betas[0]), float(betas[1]), float(eps)
        for c in range(6):
            o.wc[c] = float(wc[c])
        o.beta_pair = float(beta_pair)
        o.step = int(step)
        o.apply = int(apply)
        loss = C.c_double()
        self._inputs_ready()
        fn = lib.gc_mlp_train_step_noalloc if noalloc else lib.gc_mlp_train_step
        self._check(fn(self._h, C.c_void_p(pts.data_ptr()), C.c_void_p(tgt.data_ptr()), n2 // 2, C.byref(o),
                       C.byref(loss)))
        return loss.value

    def _points(self, fn, pts):
        torch = _torch()
        if not (pts.is_cuda and pts.is_contiguous() and pts.dtype == torch.float64 and pts.shape[0] == 3):
            raise TypeError("pts must be a contiguous float64 device tensor [3, n]")
        n = int(pts.shape[1])
        out = torch.empty((n, 12), dtype=torch.float64, device=pts.device)
        self._inputs_ready()
        self._check(fn(self._h, C.c_void_p(pts.data_ptr()), n, C.c_void_p(out.data_ptr())))
        self._outputs_ready(out, pts)
        return out

    def mlp_eval(self, pts):
        """Neural field at points (device float64 [3, n]) -> [n, 12]."""
        return self._points(lib.gc_mlp_eval, pts)

    def field_sample(self, pts):
        """Trilinear grid field at points (device float64 [3, n]) -> [n, 12]."""
        return self._points(lib.gc_field_sample, pts)

    def gather_probe(self, dt: float, n_steps: int):
        """Gather-only pass over the live particles (gc_gather_probe); returns the
        per-slot checksums (device float64)."""
        torch = _torch()
        sink = torch.empty(max(self.count(), 1), dtype=torch.float64, device=f"cuda:{self.device}")
        self._inputs_ready()
        self._check(lib.gc_gather_probe(self._h, float(dt), int(n_steps), C.c_void_p(sink.data_ptr())))
        self._outputs_ready(sink)
        return sink

    def copy_probe(self, dst, src, n_bytes: int):
        self._inputs_ready()
        self._check(lib.gc_copy_probe(self._h, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), int(n_bytes)))
        self._outputs_ready(dst, src)


def state_to_numpy(state: Dict[str, "object"]) -> Dict[str, np.ndarray]:
    out = {}
    for k, t in state.items():
        a = t.cpu().numpy()
        out[k] = a.view(np.uint32) if a.dtype == np.int32 else a
    return out
