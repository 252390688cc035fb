"""Seeded synthetic detector events for the Hough-transform tracker.

This package is input generation only: a toy barrel detector, helix tracks,
smearing and uniform noise.  It holds none of the tracker's own arithmetic
(no offset tables, no binning, no voting, no peak rule); both the CPU oracle
and the GPU path are fed from here.
"""
from .configs import CONFIGS, DETECTOR_R_MM, B_TESLA, grid_spec, workload
from .events import (EventBatch, gen_event, gen_batch, gen_config,
                     track_hits, arrival_times, concat_events)

__all__ = ["CONFIGS", "DETECTOR_R_MM", "B_TESLA", "grid_spec", "workload",
           "EventBatch", "gen_event", "gen_batch", "gen_config", "track_hits",
           "arrival_times", "concat_events"]
