"""MI355X (gfx950) library for the hot path of the augmented tree tensor
network ground-state search: rotated TPO build, effective-operator updates,
H_eff matvec, local Lanczos eigensolve, QR isometrisation and sweeps.

The compute path is the C library ``libattn.so`` (hand-written HIP kernels);
``_lib`` marshals arguments into it and ``AttnHandle`` is a small convenience
wrapper around one handle.
"""
from __future__ import annotations

import numpy as np

from . import _lib
from ._lib import (ATTN_F64, ATTN_F32, ATTN_BF16X2, ATTN_DE_STRICT, ATTN_HOST_ONLY, ATTN_DRYRUN,
                   ATTN_SOLVER_LANCZOS, ATTN_SOLVER_DAVIDSON, ATTN_PRECOND_JACOBI,
                   ATTN_PRECOND_LEARNED, ATTN_MLP_PARAMS, AttnError, solver_opts, de_opts)


class AttnHandle:
    """One problem instance on one device (owns an attn_handle)."""

    def __init__(self, problem, flags=0, device=0):
        nsites, sites, ops, coef = problem.flat_terms()
        self.problem = problem
        self.h = _lib.attn_build_tpo(problem.n_sites, problem.d, problem.m, problem.leaf_order,
                                     nsites, sites, ops, coef,
                                     np.asarray(problem.de_sites, dtype=np.int32).reshape(-1, 2),
                                     problem.de_u, flags=flags, device=device)
        self.n_nodes, self.root, self.env_bytes = _lib.attn_tree_info(self.h)

    def close(self):
        if self.h:
            _lib.attn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def node_info(self, n):
        return _lib.attn_node_info(self.h, n)

    def init_state(self, raw=None, stream=None):
        raw = self.problem.raw_concat() if raw is None else raw
        _lib.attn_init_state(self.h, raw, stream)

    def get_tensor(self, n):
        return _lib.attn_get_tensor(self.h, n)

    def set_tensor(self, n, t):
        _lib.attn_set_tensor(self.h, n, t)

    @property
    def center(self):
        return _lib.attn_get_center(self.h)

    def move_center(self, target, stream=None):
        _lib.attn_move_center(self.h, target, stream)

    def isometrize(self, frm, to, stream=None):
        _lib.attn_isometrize(self.h, frm, to, stream)

    def update_env(self, node, leg, stream=None):
        _lib.attn_update_env(self.h, node, leg, stream)

    def heff_apply(self, node, x, y, dtype=ATTN_F64, stream=None):
        """x, y: torch tensors on the handle's device (float64 for ATTN_F64,
        float32 otherwise), M elements each."""
        _lib.attn_heff_apply(self.h, node, dtype, x.data_ptr(), y.data_ptr(), stream)

    def eigsolve(self, node, opts=None, stream=None):
        return _lib.attn_eigsolve_node(self.h, node, opts, stream)

    def sweep(self, n_sweeps, opts=None, use_graphs=False):
        return _lib.attn_sweep(self.h, n_sweeps, opts, use_graphs)

    def set_precond_weights(self, params):
        _lib.attn_precond_set_weights(self.h, params)

    def solver_stats(self):
        """(Davidson iterations, fallbacks to Jacobi, last residual norm, Jacobi rate)"""
        return _lib.attn_solver_stats(self.h)

    def heff_diagonal(self, node, out, stream=None):
        """out: float64 torch tensor on the device with M elements"""
        _lib.attn_heff_diagonal(self.h, node, out.data_ptr(), stream)

    def harvest(self, node, n_pairs, cg_tol=1e-10, cg_max=2000):
        """(features [n_pairs * M, 3], targets [n_pairs * M]) float32 torch
        tensors on the device, and the achieved CG residuals."""
        import torch
        M = int(np.prod(self.node_info(node)[0]))
        f = torch.empty((n_pairs * M, 3), dtype=torch.float32, device="cuda")
        t = torch.empty(n_pairs * M, dtype=torch.float32, device="cuda")
        res = _lib.attn_precond_harvest(self.h, node, n_pairs, cg_tol, cg_max, f.data_ptr(), t.data_ptr())
        return f, t, res

    def validate(self):
        _lib.attn_validate(self.h)

    def expect_products(self, items):
        """<psi_TTN| prod A |psi_TTN> for products given as [(site, op), ...]"""
        return _lib.attn_expect_products(self.h, items)

    def measure(self, items, coef=None):
        """<psi_aTTN| coef prod A |psi_aTTN> (disentanglers contracted in)"""
        return _lib.attn_measure(self.h, items, coef)

    def correlation(self, oa, ob):
        """N x N matrix <o^a_i o^b_j> of the augmented state"""
        return _lib.attn_correlation(self.h, oa, ob, self.problem.n_sites)

    def optimize_disentanglers(self, opts=None):
        """(new matrices, gate energies before, after, steps) from the current state"""
        return _lib.attn_optimize_disentanglers(self.h, len(self.problem.de_sites), self.problem.d, opts)

    def set_disentanglers(self, de_u):
        _lib.attn_set_disentanglers(self.h, de_u)

    def get_disentanglers(self):
        return _lib.attn_get_disentanglers(self.h, len(self.problem.de_sites), self.problem.d)

    def sweep_attn(self, n_sweeps, s_ttn=1, opts=None, dopts=None, use_graphs=False):
        """aTTN sweeps: from sweep s_ttn on, the layer is optimised before each sweep"""
        return _lib.attn_sweep_attn(self.h, n_sweeps, s_ttn, opts, dopts, use_graphs)

    def checkpoint(self, path):
        _lib.attn_checkpoint(self.h, path)

    def restore(self, path):
        _lib.attn_restore(self.h, path)

    def problem_hash(self):
        return _lib.attn_problem_hash(self.h)

    def sweep_history(self):
        return _lib.attn_sweep_history(self.h)

    def counters(self):
        return _lib.attn_counters(self.h)

    def profile_start(self):
        _lib.attn_profile(self.h, 1)

    def profile_stop(self, min_dim=0):
        """(ms, flops, launches) of the matvec contraction launches since start."""
        return _lib.attn_profile(self.h, 0, min_dim)



class AttnBatch:
    """Lock-step sweeps of several AttnHandle instances (borrowed: keep them
    alive and do not use them while the batch sweeps)."""

    def __init__(self, handles, krylov_k=20, precision=ATTN_F32, use_graphs=True, autotune=False,
                 persistent=0):
        """persistent: 0 staged launches, 1 one persistent launch per matvec,
        2 per step whichever of the two timed faster at creation."""
        self.handles = list(handles)
        self.b = _lib.attn_batch_create([a.h for a in self.handles], krylov_k, precision,
                                        use_graphs, autotune, persistent)

    def sweep(self, n_sweeps):
        """(energies [n_instances][n_sweeps], seconds [n_sweeps])"""
        return _lib.attn_batch_sweep(self.b, len(self.handles), n_sweeps)

    def info(self):
        return _lib.attn_batch_info(self.b)

    def forms(self):
        """(steps that run matvecs, steps among them on the persistent launch)"""
        return _lib.attn_batch_forms(self.b)

    def close(self):
        if self.b:
            _lib.attn_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_train(feats, targets, params, steps=2000, batch=4096, lr=1e-3):
    """Train the correction model on device tensors (feats [n, 3], targets [n],
    float32); returns (params, per-step batch losses)."""
    n = int(targets.numel())
    return _lib.attn_mlp_train(feats.data_ptr(), targets.data_ptr(), n, steps, batch, lr, params)


def mlp_eval(params, feats):
    import torch
    out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
    _lib.attn_mlp_eval(params, feats.data_ptr(), out.data_ptr(), int(feats.shape[0]))
    return out
