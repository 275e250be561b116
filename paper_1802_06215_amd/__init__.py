"""hdx: DESPOT leaf-node expansion (HyP-DESPOT, Sec. III-D) on MI355X.

The compute path is the C ABI of ``libhdx.so`` (include/hdx.h) over
hand-written HIP kernels for gfx950; this package is its thin binding.
"""
from .hdx import (EXPORTS, Batch, Mlp, features, PEDNAV, POLICY_CONST, POLICY_DEFAULT, POLICY_RANDOM, ROCKSAMPLE, Context,
                  HdxError, LeafBuffers, Model, Tree, empty_states, load_library, make_leaf,
                  rollout_cfg, states_view)

__all__ = ["Batch", "Mlp", "features", "Context", "Model", "Tree", "LeafBuffers", "HdxError", "make_leaf", "rollout_cfg",
           "empty_states", "states_view", "load_library", "EXPORTS", "ROCKSAMPLE", "PEDNAV",
           "POLICY_DEFAULT", "POLICY_CONST", "POLICY_RANDOM"]
