"""torch.autograd.Function around the smooth event-count surrogate.

Forward and backward run in libevis's HIP kernels (evis_soft_count_forward
/ _backward); torch only provides the tensors and the optimiser around them.
"""
from __future__ import annotations

import torch

from . import evis


class EvisSoftCount(torch.autograd.Function):
    """S[n, H, W] = sum_j sigmoid((|L_j - R_{j-1}| - C[n]) / tau) for a batch
    of n keyframe pairs of one size; differentiable in L_A, L_B, m_A, m_B, C.

    Inputs: L_A, L_B, Z_A, Z_B, L_ref [n, H, W]; m_A, m_B [n, H, W, 2];
    C [n]; K, tau, blend_mode; ectx an evis.Context; hold_ref: treat the
    hard reference trajectory as a constant in dS/dC (EVIS_SOFT_HOLD_REF).
    """

    @staticmethod
    def forward(fctx, L_A, L_B, m_A, m_B, C, Z_A, Z_B, L_ref, K, tau, blend_mode, ectx, hold_ref=False):
        args = [t.contiguous() for t in (L_A, L_B, m_A, m_B, C, Z_A, Z_B, L_ref)]
        L_A, L_B, m_A, m_B, C, Z_A, Z_B, L_ref = args
        S = torch.empty_like(L_A)
        envs = evis.soft_env_array(L_A, L_B, m_A, m_B, Z_A, Z_B, L_ref, S=S)
        evis.evis_soft_count_forward(ectx, envs, int(K), float(tau), int(blend_mode), C)
        fctx.save_for_backward(*args)
        fctx.K, fctx.tau, fctx.blend_mode, fctx.ectx = int(K), float(tau), int(blend_mode), ectx
        fctx.flags = evis.EVIS_SOFT_HOLD_REF if hold_ref else 0
        return S

    @staticmethod
    def backward(fctx, gS):
        L_A, L_B, m_A, m_B, C, Z_A, Z_B, L_ref = fctx.saved_tensors
        gS = gS.contiguous()
        gL_A = torch.empty_like(L_A)
        gL_B = torch.empty_like(L_B)
        gm_A = torch.empty_like(m_A)
        gm_B = torch.empty_like(m_B)
        gC = torch.empty_like(C)
        envs = evis.soft_env_array(L_A, L_B, m_A, m_B, Z_A, Z_B, L_ref, gS=gS, gL_A=gL_A, gL_B=gL_B,
                                   gm_A=gm_A, gm_B=gm_B)
        evis.evis_soft_count_backward(fctx.ectx, envs, fctx.K, fctx.tau, fctx.blend_mode, C, gC,
                                      fctx.flags)
        return gL_A, gL_B, gm_A, gm_B, gC, None, None, None, None, None, None, None, None


def soft_count(L_A, L_B, m_A, m_B, C, Z_A, Z_B, L_ref, K, tau, blend_mode, ectx, hold_ref=False):
    return EvisSoftCount.apply(L_A, L_B, m_A, m_B, C, Z_A, Z_B, L_ref, K, tau, blend_mode, ectx, hold_ref)
