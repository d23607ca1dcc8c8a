"""MI355X-native batched forward dynamics of articulated apple trees.

The native library (liborchard.so, HIP for gfx950) is loaded lazily by
``load_library``/``Model``; it must be built first (``__graft_entry__.build``).
"""
from .orchard import (EVENT_BREAK, EVENT_DETACH_PULL, EVENT_DETACH_TENSION, EXPORTS, Model, OrchardError, State,
                      load_library)

from .autograd import rollout, tips

__all__ = ["rollout", "tips", "Model", "State", "load_library", "OrchardError", "EXPORTS", "EVENT_BREAK", "EVENT_DETACH_PULL",
           "EVENT_DETACH_TENSION"]
