"""Helpers shared by the GPU parity tests (not collected as tests)."""

import numpy as np

from oracle import evaluate, rsvd as orsvd


def to_np(t):
    return t.detach().cpu().numpy()


def compare_to_oracle(A64, out_gpu, k, p, q, seed, dtype, stream_id=0, sketch="gaussian"):
    """Run the oracle on exactly the matrix the GPU read and return error figures.

    out_gpu = (U, S, V, Q) as numpy arrays.  Singular vectors are compared after
    the oracle's sign normalization; Q by its projector (any orthonormal basis
    of the same range is equally valid).
    """
    U, S, V, Q = out_gpu
    ref = orsvd.rsvd(A64, k, p, q, seed=seed, stream=stream_id, dtype=dtype, sketch=sketch)
    Uo, Vo = orsvd.normalize_signs(ref["Uk"], ref["Vk"])
    Ug, Vg = orsvd.normalize_signs(U.astype(np.float64), V.astype(np.float64))
    out = {
        "sigma_rel": float(np.max(np.abs(S - ref["Sk"]) / ref["Sk"])),
        "u_err": float(np.max(np.abs(Ug - Uo))),
        "v_err": float(np.max(np.abs(Vg - Vo))),
        "orth_q": evaluate.orthonormality_error(Q.astype(np.float64)),
        "res_q": evaluate.residual_q(A64, Q.astype(np.float64)),
        "res_q_ref": evaluate.residual_q(A64, ref["Q"]),
        "res_k": evaluate.residual_usv(A64, U.astype(np.float64), S.astype(np.float64), V.astype(np.float64)),
        "res_k_ref": evaluate.residual_usv(A64, ref["Uk"], ref["Sk"], ref["Vk"]),
        "ref": ref,
    }
    return out
