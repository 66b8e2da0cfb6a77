"""torch.autograd.Function over the device entry point of libdpk.

Forward evaluates E, F and the virial in one call of the HIP path (the adjoint runs eagerly, as
the force is part of the result) and saves F. Backward returns dE/dr = -F times the incoming
gradient of E (Sec. II.A.2: F = -dE/dr). Forces and virial are returned as non-differentiable
outputs; second derivatives are not provided. PyTorch supplies only device memory and the stream.
"""
from __future__ import annotations

import torch

from . import dpk


class DPEnergyFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, coord, atype, box, context):
        n = coord.shape[0]
        dev = coord.device
        energy = torch.zeros(1, dtype=torch.float64, device=dev)
        force = torch.empty((n, 3), dtype=torch.float64, device=dev)
        virial = torch.empty((3, 3), dtype=torch.float64, device=dev)
        # waits for the frame: device-side errors (atom types out of range, a candidate buffer
        # overflowed in a locally dense spot, which is rerun with the largest buffer) are raised
        # here instead of returning wrong values
        context.compute_device_checked(coord.detach().contiguous(), atype, box, energy, force, virial)
        fctx.save_for_backward(force)
        fctx.mark_non_differentiable(force, virial)
        return energy, force, virial

    @staticmethod
    def backward(fctx, g_energy, g_force, g_virial):
        (force,) = fctx.saved_tensors
        grad = None
        if fctx.needs_input_grad[0]:
            grad = -force * g_energy.reshape(1, 1)
        return grad, None, None, None


class DPEnergy(torch.nn.Module):
    """E(coord) for a fixed atom typing and cell; call returns (E [1], F [N,3], Xi [3,3])."""

    def __init__(self, model: dpk.Model, precision: str = "mixed", device: int = 0):
        super().__init__()
        self.context = dpk.Context(model, device=device, precision=precision)

    def forward(self, coord: torch.Tensor, atype: torch.Tensor, box=None):
        if coord.dtype != torch.float64 or not coord.is_cuda:
            raise ValueError("coord must be a float64 CUDA tensor")
        if atype.dtype != torch.int32:
            atype = atype.to(torch.int32)
        return DPEnergyFunction.apply(coord, atype.contiguous(), box, self.context)
