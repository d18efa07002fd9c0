"""Batches of independent NUFFT calls (kbn_batch_* of the C ABI).

A batch is a list of tasks, each one single-plan call with its tensors.
The library runs the tasks of different plans concurrently on its own
streams and can record the whole batch into one HIP graph, replayed by
``launch()``.  This module only marshals arguments; the tensors given to a
task are kept referenced for the life of the batch because a captured
graph keeps reading and writing the same memory.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional

import torch

from . import _lib
from ._lib import check
from .nufft import KbNufft, _ptr, _stream

FORWARD = _lib.KBN_TASK_FORWARD
ADJOINT = _lib.KBN_TASK_ADJOINT
JAC_OMEGA_FWD = _lib.KBN_TASK_JAC_OMEGA_FWD
JAC_OMEGA_ADJ = _lib.KBN_TASK_JAC_OMEGA_ADJ
JAC_X_FWD = _lib.KBN_TASK_JAC_X_FWD
JAC_X_ADJ = _lib.KBN_TASK_JAC_X_ADJ


class Task:
    """One call: ``plan.<op>(a, [g,] smaps) -> out`` with B images and C coils."""

    def __init__(self, plan: KbNufft, op: int, B: int, C: int, a: torch.Tensor,
                 out: torch.Tensor, smaps: Optional[torch.Tensor] = None,
                 g: Optional[torch.Tensor] = None, accumulate: bool = False):
        for t in (a, out, smaps, g):
            if t is not None and (not t.is_contiguous() or t.device != plan.device):
                raise ValueError("task tensors must be contiguous and on the plan's device")
        self.plan, self.op, self.B, self.C = plan, int(op), int(B), int(C)
        self.a, self.out, self.smaps, self.g = a, out, smaps, g
        self.accumulate = bool(accumulate)

    def struct(self) -> _lib.KbnTask:
        t = _lib.KbnTask()
        t.plan = self.plan._h
        t.op = self.op
        t.B = self.B
        t.C = self.C
        t.a = _ptr(self.a)
        t.smaps = _ptr(self.smaps)
        t.g = _ptr(self.g)
        t.out = _ptr(self.out)
        t.accumulate = int(self.accumulate)
        return t


class KbnBatch:
    """``fuse=True``: interpolation of all tasks in one launch per phase and
    kernel shape (kbn_batch_fuse); the tasks must then be independent."""

    def __init__(self, tasks: List[Task], nstreams: int = 0, fuse: bool = False):
        if not tasks:
            raise ValueError("empty task list")
        self.tasks = list(tasks)
        self.device = tasks[0].plan.device
        arr = (_lib.KbnTask * len(tasks))(*[t.struct() for t in tasks])
        h = ctypes.c_void_p()
        check(_lib.lib().kbn_batch_create(ctypes.byref(h), len(tasks), arr, int(nstreams)),
              "kbn_batch_create")
        self._h = h
        if fuse:
            check(_lib.lib().kbn_batch_fuse(self._h, 1), "kbn_batch_fuse")

    def run(self):
        """Issue every task once on the current stream's timeline."""
        check(_lib.lib().kbn_batch_run(self._h, _stream(self.device)), "kbn_batch_run")

    def capture(self):
        """Run once, then record the batch into a graph for launch()."""
        check(_lib.lib().kbn_batch_capture(self._h, _stream(self.device)), "kbn_batch_capture")

    def launch(self):
        check(_lib.lib().kbn_batch_launch(self._h, _stream(self.device)), "kbn_batch_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().kbn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
