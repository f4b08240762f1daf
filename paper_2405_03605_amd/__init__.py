"""MI355X-native island-model GA generation step (HIP kernels behind a C ABI).

Import is light: the HIP library is loaded on first use of GARun / GABatch.
"""
from ._lib import (ASYNC_UNPACED, FORM_AUTO, FORM_RESIDENT, FORM_STREAMING, MODEL_FITNESS,
                   MODEL_ONEMAX, MODEL_TRAP4, POLICY_HYBRID, POLICY_STEADY, POLICY_TILTED,
                   SCHEDULE_ASYNC,
                   SCHEDULE_SYNC, GAError, build, load)
from .run import CONFIG_FIELDS, GABatch, GAPool, GARun, state_bytes

__all__ = ["GARun", "GABatch", "GAPool", "GAError", "build", "load", "state_bytes", "CONFIG_FIELDS",
           "FORM_AUTO", "FORM_STREAMING", "FORM_RESIDENT", "SCHEDULE_SYNC", "SCHEDULE_ASYNC",
           "ASYNC_UNPACED", "MODEL_FITNESS", "MODEL_ONEMAX", "MODEL_TRAP4", "POLICY_STEADY",
           "POLICY_TILTED", "POLICY_HYBRID"]
