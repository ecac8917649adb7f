"""Shared helpers for the GPU parity tests: build operators through the C ABI and the matching
oracle operators on the same seeded inputs."""
import numpy as np

import vsie_synth as synth
from oracle import system, tt


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def oracle_same(problem, op, tt_eps=1e-4, pc_dist=2):
    """Oracle O_same with the oracle's own TT-SVD cores and SVD low-rank factors, imported into
    the library so that both apply the identical compressed operator."""
    d = system.discretize(problem)
    S_direct, blocks = system.assemble_direct(d)
    cores = None
    aca = None
    if d.far is not None:
        cores = [tt.tt_svd(system.far_coupling_tensor(d, a), tt_eps) for a in range(3)]
        for a in range(3):
            op.import_tt(a, cores[a])
        if d.near is not None:
            U, sv, Vh = np.linalg.svd(blocks["nf"], full_matrices=False)
            r = int(min(256, np.sum(sv > 1e-9 * sv[0])))
            aca = (U[:, :r] * sv[:r], Vh[:r].conj().T)
            op.import_aca(*aca)
    S_same, _, parts = system.assemble_same(d, cores, aca, pc_dist, direct_blocks=blocks)
    return d, S_direct, S_same, parts


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def far_shield_case():
    """8^3 body, loop, and a distant closed shield (low TT rank) for TT-cross accuracy tests."""
    g = synth.sphere_phantom((8, 8, 8), 5e-3, 17e-3, 52.0, 0.55)
    loop = synth.strip_loop_flat((25.5e-3, 0.37e-3, -0.41e-3), side=30e-3, width=5e-3, step=5e-3)
    shield = synth.cylinder_shield(0.200, 0.400, 24, 12, closed=True, cap_rings=2)
    return synth.Problem(g, [shield, loop], synth.problems.LARMOR_7T_HZ, "far-shield")
