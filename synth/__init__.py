"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package only draws random inputs (cell layouts, embeddings, masks).  It
holds none of the clustering method's arithmetic, so both the oracle and the
GPU path can consume its frames without sharing any of the method's code.
"""
from .frames import (FrameSpec, Frame, make_frame, TINY, PLAIN512, PRECISION1024,
                     MID, batch_specs, drifting_sequence, circle_points, blob_points, overlap_circles)

__all__ = ["FrameSpec", "Frame", "make_frame", "TINY", "PLAIN512", "PRECISION1024", "MID",
           "batch_specs", "drifting_sequence", "circle_points", "blob_points", "overlap_circles"]
