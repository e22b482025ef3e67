"""torch.autograd.Function over libtmm's discrete adjoint.

``TMMYearMisfit.apply(u, y0, handle, obs)`` returns the least-squares misfit
J (one value per ensemble member) of one model year started from y0 with
parameters u, against month-end observations obs.  Its backward pass
returns dJ/du and dJ/dy0 computed by ``tmm_year_adjoint``: the checkpointed
adjoint sweep runs in the HIP library, this class only moves the results.
Sections 1.2, 6.1 and 9 of the paper name exact derivatives by algorithmic
differentiation as the route to sensitivities and parameter optimisation.
"""

import numpy as np
import torch


class TMMYearMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, y0, handle, obs):
        """u: (nbatch, nparam) float64 tensor (any device); y0: (n, W) CUDA
        float64; handle: a ``tmm.TMM`` with an adjoint-capable workspace;
        obs: (nmat, n, W) CUDA float64.  Returns J as a (nbatch,) tensor on
        u's device."""
        uu = np.atleast_2d(u.detach().cpu().numpy().astype(np.float64))
        handle.set_params(uu)
        J, G, dy0 = handle.year_adjoint(y0.detach().contiguous(), obs, want_dy0=True)
        ctx.save_for_backward(torch.as_tensor(G, dtype=u.dtype, device=u.device), dy0)
        ctx.u_shape = u.shape
        return torch.as_tensor(J, dtype=u.dtype, device=u.device)

    @staticmethod
    def backward(ctx, gJ):
        G, dy0 = ctx.saved_tensors
        gu = (gJ.reshape(-1, 1) * G).reshape(ctx.u_shape)
        gy0 = None
        if ctx.needs_input_grad[1]:
            # dJ_b/dy0 for every member is packed in the member's state columns
            nb = G.shape[0]
            ntr = dy0.shape[1] // nb
            scale = gJ.detach().to(dy0.device).repeat_interleave(ntr)
            gy0 = dy0 * scale.reshape(1, -1)
        return gu, gy0, None, None


def year_misfit(u, y0, handle, obs):
    """Functional form of :class:`TMMYearMisfit`."""
    return TMMYearMisfit.apply(u, y0, handle, obs)
