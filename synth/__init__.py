"""Seeded synthetic inputs for the Voronoi ray walk.

This package is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests. It produces inputs only (site clouds, the Delaunay neighbour
CSR built by a CPU builder, per-cell attributes, camera poses, upstream
gradients, serving request streams). It holds none of the walk's arithmetic:
no ray/plane intersection, no compositing, no spherical harmonics, no ray
generation.
"""

from .scenes import (  # noqa: F401
    CONFIGS,
    Camera,
    Scene,
    build_adjacency,
    make_cameras,
    make_scene,
    make_upstream_grads,
    make_serving_requests,
    nearest_site,
    small_scene,
)
