"""MI355X (gfx950) induced-dipole solver of a Thole-damped point-dipole polarizable force field:
PCG on (alpha^-1 - T) mu = E_perm with a blocked real-space tile kernel and smooth PME, in FP64
or mixed precision (FP32 math, 64-bit fixed-point fields, FP64 PCG).

The compute path is libamoeba.so (HIP, C ABI in include/amoeba.h); `amoeba` is its ctypes
binding and `synth` the seeded workload generators."""
__all__ = ["amoeba", "synth"]
