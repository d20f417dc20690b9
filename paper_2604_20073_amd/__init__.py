"""Worst-case-optimal Datalog on AMD MI355X (gfx950).

The engine lives in ``libwcdl.so`` (HIP kernels + C ABI, include/wcdl.h);
``engine.Engine`` is its Python binding.
"""

from .engine import (WCDL_F_BALANCE_OFF, WCDL_F_BATCHED, WCDL_F_CHECKED, WCDL_F_COST_PLANNER,
                     WCDL_F_GROUPED_SORT_OFF, WCDL_F_HEAD_BODY_OFF, WCDL_F_RUN_BITMAPS_OFF,
                     WCDL_F_STAGE_OFF, WCDL_F_STREAMS_OFF, WCDL_F_TILE_DEDUP_OFF, WCDL_F_XPROD_OFF,
                     Engine, Instance, WcdlError, decode_unit, owner_key, work_slice)

__all__ = ["Engine", "Instance", "WcdlError", "work_slice", "owner_key", "decode_unit",
           "WCDL_F_BALANCE_OFF", "WCDL_F_STREAMS_OFF", "WCDL_F_XPROD_OFF", "WCDL_F_STAGE_OFF",
           "WCDL_F_BATCHED", "WCDL_F_HEAD_BODY_OFF", "WCDL_F_RUN_BITMAPS_OFF",
           "WCDL_F_GROUPED_SORT_OFF", "WCDL_F_CHECKED", "WCDL_F_COST_PLANNER",
           "WCDL_F_TILE_DEDUP_OFF"]
