"""Seeded synthetic inputs: detector description and cluster sets."""
from . import geometry
from .events import (ClusterSet, RadialDistortion, Tracks, build_clusters, central_event,
                     exact_tracks, helix_crossings, single_sector, slice_batch_collisions,
                     timeframe_slice)

__all__ = ["geometry", "ClusterSet", "RadialDistortion", "Tracks", "build_clusters",
           "central_event", "exact_tracks", "helix_crossings", "single_sector",
           "slice_batch_collisions", "timeframe_slice"]
