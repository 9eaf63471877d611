"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the DG update: it builds meshes and projects analytic
initial fields onto the P1 representation, once, on the host.  Both the GPU path
and the CPU oracle receive the arrays it returns.

State layout (coefficient-major, ``U[k * ncells + cell]``):
  * hydro variable ``v`` (rho, rho v_x, rho v_y[, rho v_z], E) owns the arrays
    ``k = v*(1+dim) + c`` with ``c = 0`` the cell mean and ``c = 1..dim`` the
    gradient along x, y(, z) about the centroid (the Taylor basis of Sec. 2.2);
  * ideal MHD (3D) appends the three B means and then the coefficients
    a4..a11 of the divergence-free functions V4..V11 of Sec. 2.2.
Cells are numbered x fastest: ``cell = (k*Ny + j)*Nx + i``.
"""
from __future__ import annotations

import numpy as np

from .cartesian import (acoustic_state, alfven2d_state, alfven_state, batched_instances,
                        batched_state, c1_state, c2_state, orszag_tang_state, rotor_state,
                        c3_state, cartesian_centres, gresho_state, project_cartesian,
                        random_p1_state, vortex_cell_means, vortex_fields)

__all__ = [
    "acoustic_state", "alfven2d_state", "alfven_state", "batched_instances", "batched_state",
    "orszag_tang_state", "rotor_state", "c1_state", "c2_state", "c3_state",
    "cartesian_centres", "gresho_state", "project_cartesian", "random_p1_state",
    "vortex_cell_means", "vortex_fields",
]
