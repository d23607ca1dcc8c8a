"""MI355X-native batched forward dynamics of articulated apple trees.

The native library (liborchard.so, HIP for gfx950) is loaded lazily by
``load_library``/``Model``; it must be built first (``__graft_entry__.build``).
"""
from .orchard import (DEFAULT_TUNING, EVENT_BREAK, EVENT_DETACH_PULL, EVENT_DETACH_TENSION, EXPORTS, Graph, Model,
                      OrchardError, State, autotune, load_library, sphere_fit)

from .autograd import rollout, tips

__all__ = ["rollout", "tips", "Model", "State", "Graph", "autotune", "DEFAULT_TUNING", "load_library", "OrchardError",
           "EXPORTS", "sphere_fit", "EVENT_BREAK", "EVENT_DETACH_PULL", "EVENT_DETACH_TENSION"]
