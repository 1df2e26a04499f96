"""Grouped (batched) dgemm launches: plan on the host, run as one persistent kernel.

A `GroupedPlan` takes a list of GEMMs on device tensors, checks each one's storage extents,
asks the library for a plan (descriptors + tile list), keeps the plan in device memory and
launches it. Launches allocate nothing, so they can be captured in a torch CUDA (HIP) graph.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import binding as b


class GroupedPlan:
    def __init__(self, gemms, tile_class=None, schedule=b.MDG_SCHEDULE_LPT):
        """gemms: dicts with transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc
        (A, B, C float64 device tensors or addresses); tile_class: per-GEMM list or None."""
        import torch
        descs = []
        for g in gemms:
            (ta, tb, m, n, k, alpha, pa, lda, pb, ldb, beta, pc, ldc, _) = b._marshal(
                g["transa"], g["transb"], g["m"], g["n"], g["k"], g["alpha"], g["A"], g["lda"],
                g["B"], g["ldb"], g["beta"], g["C"], g["ldc"], None)
            descs.append(b.mdg_gemm_desc(ta, tb, m, n, k, alpha, pa, lda, pb, ldb, beta, pc, ldc))
        self.count = len(descs)
        self.tile_class = None if tile_class is None else [int(c) for c in tile_class]
        nbytes = b.mdg_grouped_plan_bytes(descs, self.tile_class)
        if nbytes < 0:
            raise ValueError("invalid grouped plan request (tile classes?)")
        host = np.zeros(nbytes, dtype=np.uint8)
        st, self.num_tiles, bad = b.mdg_grouped_plan(descs, self.tile_class, schedule, host)
        if st:
            raise b.MdgError(st) if st < 100 else ValueError(
                f"GEMM {bad}: {b.mdg_status_string(st - 100)}")
        self.host_plan = host
        self.device_plan = torch.from_numpy(host).to("cuda")
        self._gemms = gemms  # keeps the operand tensors alive with the plan

    def launch(self, grid=0, stream=None):
        st = b.mdg_dgemm_grouped(self.device_plan, self.num_tiles, grid, stream)
        if st:
            raise b.MdgError(st)
