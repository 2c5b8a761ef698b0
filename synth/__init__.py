"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle.

This package only *describes problems*: meshes, material fields, boundary
sets, traction values, warm-start noise and arrival times.  It holds none of
the finite-element arithmetic (no shape functions, no stresses, no energies,
no solvers), so the oracle and the device path can both consume it without
sharing any of the method.

Every generator takes an explicit integer seed and uses
``numpy.random.Generator(PCG64(seed))``.
"""
from .problems import (Problem, MODELS, unit_square_c1, plate_problem,
                       box_problem, c4_member, batch_c4, serving_stream,
                       serving_problem, structured_plate, structured_box,
                       beam_problem, cook_problem,
                       SERVING_E_FEATURES, SERVING_NOISE_FEATURES)
from .fields import rff_field, lifting_weight, warm_start_guess, warm_start_noise

__all__ = ["Problem", "MODELS", "unit_square_c1", "plate_problem",
           "box_problem", "c4_member", "batch_c4", "serving_stream",
           "serving_problem", "structured_plate",
           "structured_box", "beam_problem", "cook_problem", "rff_field", "lifting_weight",
           "warm_start_guess", "warm_start_noise", "SERVING_E_FEATURES",
           "SERVING_NOISE_FEATURES"]
