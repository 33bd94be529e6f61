"""MI355X (gfx950) VGICP matching-cost library: voxel maps, factor linearization (unary 6x6 and
binary 12x12), evaluation, batched persistent linearization under HIP graphs, and the
hand-written backward pass (Koide et al., ICRA 2022, Sec. III-A, Eqs. (2)-(3)).

The compute lives in libvgicp.so (include/vgicp.h); ``paper_2202_00242_amd.vgicp`` binds it and
``paper_2202_00242_amd.autograd`` wraps it for torch.autograd. Importing those submodules
requires the built library.
"""
__all__ = ["vgicp", "autograd", "build"]
