"""Batched persistent decoding of several codes in one launch (ldpc_decode_multi),
captured plans (ldpc_plan_*), and the launch-shape autotuner (ldpc_autotune_multi)."""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

import torch

from ._lib import check, lib, stream_handle
from .graph import Graph

MAX_CODES = 8


class Job(ctypes.Structure):
    _fields_ = [("llr", ctypes.c_void_p), ("batch", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("hard_bits", ctypes.c_void_p), ("posterior", ctypes.c_void_p), ("iters_used", ctypes.c_void_p)]


STREAM_AUTO = 0xFFFFFFFF  # every code whose word state fits LDS runs in the stream form
SPLIT_AUTO = 0xFFFFFFFF  # every other code with fewer 64-word tiles than half the compute units: split form


class Shape(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("slots", ctypes.c_int32 * MAX_CODES), ("refill", ctypes.c_int32),
                ("stream_codes", ctypes.c_uint32), ("split_codes", ctypes.c_uint32), ("lanes", ctypes.c_int32),
                ("stream_threads", ctypes.c_int32 * MAX_CODES), ("split_slices", ctypes.c_int32 * MAX_CODES),
                ("span", ctypes.c_int32 * MAX_CODES)]

    @classmethod
    def make(cls, waves=0, slots=None, refill=0, stream_codes=0, split_codes=0, lanes=0, stream_threads=None,
             split_slices=None, span=None):
        s = cls()
        for i, v in enumerate(span or []):
            s.span[i] = int(v)
        s.waves = int(waves)
        s.refill = int(refill)
        s.lanes = int(lanes)
        for i, v in enumerate(stream_threads or []):
            s.stream_threads[i] = int(v)
        for i, v in enumerate(split_slices or []):
            s.split_slices[i] = int(v)
        s.stream_codes = int(stream_codes) & 0xFFFFFFFF
        s.split_codes = int(split_codes) & 0xFFFFFFFF
        for i, v in enumerate(slots or []):
            s.slots[i] = int(v)
        return s

    def as_dict(self, ncodes):
        d = {"waves": self.waves, "slots": [self.slots[i] for i in range(ncodes)], "refill": self.refill,
             "lanes": self.lanes, "stream_threads": [self.stream_threads[i] for i in range(ncodes)],
             "split_slices": [self.split_slices[i] for i in range(ncodes)],
             "span": [self.span[i] for i in range(ncodes)]}
        if self.stream_codes:
            d["stream_codes"] = [i for i in range(ncodes) if (self.stream_codes >> i) & 1]
        if self.split_codes:
            d["split_codes"] = [i for i in range(ncodes) if (self.split_codes >> i) & 1]
        return d


FAULT_OFFSET = 480  # LDPC_MULTI_FAULT_OFFSET


def fault(workspace: torch.Tensor) -> int:
    """The fault word of the last batched launch on this workspace: nonzero iff a group
    slot's barrier gave up waiting (its outputs are then invalid).  Synchronises."""
    return int(workspace[FAULT_OFFSET:FAULT_OFFSET + 4].view(torch.int32).item())


class Batch:
    """Inputs, outputs and device arrays of one batched decode (pointers fixed for plans)."""

    def __init__(self, graphs, llrs, max_iters, orders=None):
        if not 1 <= len(graphs) <= MAX_CODES or len(llrs) != len(graphs):
            raise ValueError("need 1..8 codes with one llr tensor each")
        if isinstance(max_iters, int):
            max_iters = [max_iters] * len(graphs)
        self.graphs = list(graphs)
        self.llrs = []
        self.outs = []
        for g, x in zip(graphs, llrs):
            if not x.is_cuda or x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != g.n:
                raise ValueError("llr must be a cuda float32 tensor [B, n]")
            x = x.contiguous()
            B = x.shape[0]
            self.llrs.append(x)
            self.outs.append((torch.empty((B, g.n), dtype=torch.uint8, device=x.device),
                              torch.empty((B, g.n), dtype=torch.float32, device=x.device),
                              torch.empty((B,), dtype=torch.int32, device=x.device)))
        n = len(graphs)
        self.ncodes = n
        self._gh = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
        self._jobs = (Job * n)()
        for i, (x, (h, p, it)) in enumerate(zip(self.llrs, self.outs)):
            self._jobs[i] = Job(x.data_ptr(), x.shape[0], int(max_iters[i]), h.data_ptr(), p.data_ptr(),
                                it.data_ptr())
        self.orders = None
        self._orders = None
        if orders is not None:
            self.orders = [None if o is None else o.to(dtype=torch.int32).contiguous() for o in orders]
            self._orders = (ctypes.c_void_p * n)(*[0 if o is None else o.data_ptr() for o in self.orders])

    def resolve(self, shape: Shape | None = None):
        out = Shape()
        nb = ctypes.c_size_t()
        check("ldpc_multi_resolve", lib().ldpc_multi_resolve(self._gh, self.ncodes, self._jobs,
                                                             ctypes.byref(shape) if shape else None,
                                                             ctypes.byref(out), ctypes.byref(nb)))
        return out, nb.value

    def workspace(self, shape: Shape | None = None) -> torch.Tensor:
        _, nb = self.resolve(shape)
        return torch.empty((max(nb, 256),), dtype=torch.uint8, device=self.llrs[0].device)

    def run(self, early_stop=True, shape: Shape | None = None, workspace=None, stream=None):
        if workspace is None:
            workspace = self.workspace(shape)
        check("ldpc_decode_multi",
              lib().ldpc_decode_multi(self._gh, self.ncodes, self._jobs, self._orders, int(bool(early_stop)),
                                      ctypes.byref(shape) if shape else None, ctypes.c_void_p(workspace.data_ptr()),
                                      workspace.numel(), ctypes.c_void_p(stream_handle(stream))))
        return self.outs

    def autotune(self, early_stop=True, stream=None, persistent_only=False):
        """ldpc_autotune_multi: the fastest shape (forms per code and launch shapes) and its time."""
        best = Shape()
        ms = ctypes.c_float()
        check("ldpc_autotune_multi",
              lib().ldpc_autotune_multi(self._gh, self.ncodes, self._jobs, self._orders, int(bool(early_stop)),
                                        1 if persistent_only else 0, ctypes.c_void_p(stream_handle(stream)),
                                        ctypes.byref(best), ctypes.byref(ms)))
        return best, ms.value


def decode_multi(graphs, llrs, max_iters, early_stop=True, shape=None, orders=None):
    """Decode per-code batches in one persistent launch; returns [(hard, post, iters)] per code."""
    b = Batch(graphs, llrs, max_iters, orders)
    return b.run(early_stop, shape)


class Plan:
    """A batched decode captured once into a HIP graph and replayed with ``launch()``."""

    def __init__(self, batch: Batch, early_stop=True, shape: Shape | None = None):
        self.batch = batch
        self.shape = shape
        self.ws = batch.workspace(shape)
        self._capture = torch.cuda.Stream()
        h = ctypes.c_void_p()
        check("ldpc_plan_create_multi",
              lib().ldpc_plan_create_multi(batch._gh, batch.ncodes, batch._jobs, batch._orders,
                                           int(bool(early_stop)), ctypes.byref(shape) if shape else None,
                                           ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                           ctypes.c_void_p(self._capture.cuda_stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        check("ldpc_plan_launch", lib().ldpc_plan_launch(self._h, ctypes.c_void_p(stream_handle(stream))))
        return self.batch.outs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ldpc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def _signature(graphs, batch: Batch, early_stop) -> str:
    h = hashlib.sha1()
    for g, x, j in zip(graphs, batch.llrs, batch._jobs):
        c, v = g.edge_arrays()
        h.update(c.tobytes())
        h.update(v.tobytes())
        h.update(f"{g.m},{g.n},{x.shape[0]},{j.max_iters};".encode())
    h.update(f"es={int(bool(early_stop))};{torch.cuda.get_device_properties(0).gcnArchName};shape-v4".encode())
    return h.hexdigest()


def _mask(codes) -> int:
    m = 0
    for q in codes:
        m |= 1 << int(q)
    return m


def cache_path() -> str:
    base = os.environ.get("LDPC_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ldpc_mi355x")
    return os.path.join(base, "autotune.json")


def tuned_shape(batch: Batch, early_stop=True, retune=False, persistent_only=False) -> Shape:
    """Shape for this batch from the JSON cache (per code signature, batch, iteration limits,
    early stop and GPU architecture), running the autotuner on a miss.  persistent_only keeps
    every code in the persistent launch and tunes its shape only."""
    key = _signature(batch.graphs, batch, early_stop) + (":persistent" if persistent_only else ":forms")
    path = cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache and not retune:
        d = cache[key]
        return Shape.make(d["waves"], d["slots"], d.get("refill", 0), _mask(d.get("stream_codes", [])),
                          _mask(d.get("split_codes", [])), d.get("lanes", 0), d.get("stream_threads"),
                          d.get("split_slices"), d.get("span"))
    best, ms = batch.autotune(early_stop, persistent_only=persistent_only)
    cache[key] = dict(best.as_dict(batch.ncodes), ms=ms)
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass
    return best
