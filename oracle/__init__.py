"""FP64 CPU oracle of the kinetic compressive sensing sweep.

TEST INFRASTRUCTURE ONLY.  Imported by tests/, by the smoke check and by the CPU-baseline leg
of bench.py, never by the HIP library or its Python binding.  Plain and slow on purpose: Siddon
system matrix in C (siddon.c), everything else NumPy/SciPy in FP64, each function citing the
passage of the paper it follows.
"""
from .geometry import (Geometry, build_oracle_library, forward, back, subset_angles, subset_rows,
                       subset_sensitivity, system_matrix, siddon_line)
from .model import Kinetics, cp, input_integrals, model_tac, cumulative_tissue, moments, net_influx
from .recon import (Frames, LMOptions, Prior, expected_counts, huber, huber_grad, icm, icm_sweep,
                    initial_image, initial_state, lm_fit, lm_iteration, neighbour_terms, osl_update,
                    subset_mult)
from .rebin import ssrb
from .study import Study, fitting_blood_fraction, initial_maps, make_plane_study, make_study
