"""MI355X (gfx950) unscented-transform Gaussian rasterizer for cameras and spinning LiDAR.

Every stage runs as a hand-written HIP kernel in ``libutrast.so`` behind the C-ABI of
``include/utrast.h``; this package only marshals arguments (torch supplies device memory
and streams)."""
from ._abi import LIB_PATH, UtError, lib
from .render import (ALPHA_MAX, ALPHA_MIN, T_MIN, UT_ABK, BinLists, GaussianSet, Projection, RenderOut, Sensor, SensorPipeline,
                     TileLists, Workspace, alloc_out, alloc_projection, backward, bin_and_sort, composite,
                     composite_batch, composite_batch_noalloc, lidar_tiling, project, render, render_params, tile_lists,
                     actor_poses, actor_transform, actor_transform_backward, FrameGraph, spatial_order, gather)
from .autograd import ActorTransform, UTRender, render_differentiable, transform_differentiable

__all__ = ["LIB_PATH", "UtError", "lib", "GaussianSet", "Sensor", "Projection", "TileLists", "RenderOut",
           "Workspace", "SensorPipeline", "BinLists", "tile_lists", "project", "bin_and_sort", "composite", "composite_batch", "composite_batch_noalloc", "backward", "render",
           "render_params", "alloc_out", "alloc_projection", "lidar_tiling", "UTRender",
           "render_differentiable", "ALPHA_MIN", "ALPHA_MAX", "T_MIN", "UT_ABK", "actor_poses",
           "actor_transform", "actor_transform_backward", "ActorTransform", "transform_differentiable", "FrameGraph", "spatial_order", "gather"]
