"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

Holds no arithmetic of the dynamics step (see ``treegen``)."""
from .treegen import TreeDesc, gen_tree, chain_tree, random_small_tree, ternary_lsystem_count, depth_stats
from .presets import STEP_CONSTANTS, EXTRAS_ON, EXP_STIFFNESS, step_constants, WORKLOADS, Batch, assemble, make_batch, make_trees, n_trees, pull_forces, geometry_perturbation, grad_apple_forces, grad_targets
