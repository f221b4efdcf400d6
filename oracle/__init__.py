"""FP64 CPU oracle (test infrastructure only; see oracle.py)."""
from .oracle import (Problem, State, build, compile_source, constants,  # noqa: F401
                     cpml_profile, lib, load, use_library)
