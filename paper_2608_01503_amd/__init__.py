"""MI355X-native synchronous multilevel LambdaCC clustering (pLouvain / Louvain+, pLeiden, pLeiden+).

The computation lives in the HIP library ``liblcc.so`` (hand-written gfx950 kernels behind the C-ABI of
``include/lcc.h``); :mod:`paper_2608_01503_amd.lcc` is its thin ctypes binding.
"""
from .lcc import (LCC_FLAG_LEVEL_CAP, LCC_FLAG_REFINE_NO_PROGRESS, LCC_LOUVAIN, LCC_PLEIDEN,  # noqa: F401
                  LCC_NOALLOC_SCRATCH_BYTES, LCC_PLEIDEN_PLUS, LCC_PLOUVAIN, LCC_VW_GIVEN, LCC_VW_UNIT,
                  LCC_VW_WEIGHTED_DEGREE, Context,
                  LccError, Result, Server, lcc_default_options, lcc_default_tuning, lcc_objective,
                  lcc_workspace_bytes, load,
                  make_graph, tuning_dict)
