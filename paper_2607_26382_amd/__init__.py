"""MI355X-native guarded SIMP state solve (matrix-free hex8 operator, GMG-
preconditioned FGMRES, FP64 true-residual guard, probe -> floor ladder).

The compute path is the HIP library libtopoguard.so (C ABI in
include/topoguard.h); ``topoguard`` is its torch-facing binding.
"""
