"""MI355X-native batched Pauli-frame sampler for noisy stabilizer circuits.

Implements the bulk-sampling path of Gidney, "Stim: a fast stabilizer circuit
simulator" (arXiv:2103.02202): a host-side inverse-tableau reference sample
(Sec. 4) followed by Pauli-frame propagation of many shots at once (Sec. 3,
data layout of Sec. 5.1) in hand-written HIP kernels for gfx950.

The native library (``libstimgpu.so``) is loaded lazily by
:mod:`paper_2103_02202_amd.stim_gpu`; importing this package does not touch
the GPU.
"""
