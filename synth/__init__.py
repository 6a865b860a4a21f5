"""Seeded synthetic inputs for the incremental-SVD engine and its oracle.

This package generates *inputs only*: factor-model return panels, appended
rows and columns, and update-event schedules.  It holds none of the update
method's arithmetic, so both the GPU engine's tests and the CPU oracle may
draw from it without sharing any part of the method.

All randomness is counter-based (Philox4x32-10, Salmon et al., SC'11) and
keyed by (seed, stream, purpose, tick, index): any single entry of any panel
can be regenerated on its own, on the host (numpy, here) or on the device
(``synth/csrc/synth.hip``), in any order.
"""
from .philox import philox4x32_10, uniforms, normals
from .factor_model import (FactorStream, factor_lambdas, Event, ROW, COL, ENTRY,
                           event_schedule_c0, event_schedule_iid)

__all__ = ["philox4x32_10", "uniforms", "normals", "FactorStream", "factor_lambdas",
           "Event", "ROW", "COL", "ENTRY", "event_schedule_c0", "event_schedule_iid"]
