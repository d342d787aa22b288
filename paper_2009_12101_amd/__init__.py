"""MI355X-native compressed-basis GMRES (CB-GMRES).

Restarted GMRES (Fig. 1 of Aliaga et al., "Compressed Basis GMRES on High
Performance GPUs") whose Krylov basis is stored in fp32 / fp16 / bf16 /
fp8-e4m3 / int32 / int16 and widened to FP64 in registers on every read.
The solver and every kernel of the hot path live in libcbgmres.so
(hand-written HIP for gfx950, C ABI in include/cbgmres.h); this package is
its ctypes binding plus seeded synthetic problem generators. torch supplies
device memory and streams only.
"""
from . import problems
from ._binding import (FORMATS, FORMAT_BYTES, PRECONDS, CbgError, DeviceCSR, SolveResult,
                       adam_step, basis_ld, block_jacobi_apply, block_jacobi_setup,
                       csr_transpose_values, decode, encode,
                       kernel_workspace_bytes, learned_build, learned_build_stencil, lib,
                       mlp_backward, mlp_forward, stencil_apply,
                       multidot, multidot_noalloc, NOALLOC_MAX_J, PROFILE_STRIDE, solve, spai_assemble, spai_features, spai_grad_o, spai_grad_p,
                       spai_loss_grad, spai_pack, spai_round_weights, spai_workspace_bytes, spmv,
                       strerror, update, update_redot, workspace_basis, workspace_bytes)

__all__ = ["problems", "FORMATS", "FORMAT_BYTES", "PRECONDS", "CbgError", "DeviceCSR",
           "SolveResult", "adam_step", "basis_ld", "block_jacobi_apply", "block_jacobi_setup",
           "csr_transpose_values", "decode", "encode",
           "kernel_workspace_bytes", "learned_build", "learned_build_stencil", "lib",
           "mlp_backward", "mlp_forward", "stencil_apply",
           "multidot", "multidot_noalloc", "NOALLOC_MAX_J", "PROFILE_STRIDE", "solve", "spai_assemble", "spai_features", "spai_grad_o", "spai_grad_p",
           "spai_loss_grad", "spai_pack", "spai_round_weights", "spai_workspace_bytes", "spmv",
           "strerror", "update", "update_redot", "workspace_basis", "workspace_bytes"]
