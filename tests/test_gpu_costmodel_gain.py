"""What the trained network gains over the method without it.

The method without the network picks, among the feasible leaves of the case
table, the candidate of least analytic estimate (the CASE policy).  On shapes
the float32 model never saw -- the first 100 of the 500 held-out shapes,
log-uniform on [64, 8192]^3 from seed 2 (the training shapes come from seed 1
and the 216-shape sweep) -- every feasible candidate is timed on the device
(pk_measure, the auto-tuner's measurement), and each policy's pick is scored
by those timings: ratio = t_best / t_pick.  The geometric mean of the model's
own pick (LEARNED with no measurement) must exceed CASE's, and LEARNED with
its default 5 % margin (near ties measured) must not fall below the model's
own pick.

Operands are packed prefixes of two float32 buffers (uniform on [-1, 1)
from seeds 0 and 1), as the tuner times them.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu

COUNT = 100


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def geomean(r):
    return float(np.exp(np.mean(np.log(np.asarray(r)))))


def program_key(t, p):
    # a compiled program and its split factor: the split forms of one tile
    # program share its kernel name, and two (leaf, E) points may run one
    # instance (the fastest of their timings is the program's)
    return pk.pk_kernel_name(t, p, "f32"), max(p.ks, 1)


def test_network_gains_over_case_on_heldout_shapes():
    t = pk.pk_case_table_build(0)
    assert "f32" in pk.load_shipped_models(t)
    shapes = [tuple(int(x) for x in r) for r in inputs.log_uniform_shapes(500, 2)[:COUNT]]
    big = max(max(M * K, K * N, M * N) for M, N, K in shapes)
    Abuf = inputs.uniform_f32((big,), seed=0).cuda()
    Bbuf = inputs.uniform_f32((big,), seed=1).cuda()
    Cbuf = torch.empty((big,), dtype=torch.float32, device="cuda")
    case, model, learned = [], [], []
    try:
        for (M, N, K) in shapes:
            A = Abuf[:M * K].view(M, K)
            B = Bbuf[:K * N].view(K, N)
            C = Cbuf[:M * N].view(M, N)
            times = {}
            for p, s in pk.pk_measure(t, "f32", M, N, K, A, B, C):
                k = program_key(t, p)
                times[k] = min(times.get(k, s), s)
            assert times and all(np.isfinite(v) and v > 0 for v in times.values())
            best = min(times.values())

            def score(policy):
                return best / times[program_key(t, pk.pk_select_operands(t, "f32", A, B, policy))]
            case.append(score(pk.PK_POLICY_CASE))
            pk.pk_case_table_set_learned_margin(t, 0.0)
            model.append(score(pk.PK_POLICY_LEARNED))
            pk.pk_case_table_set_learned_margin(t, 0.05)
            learned.append(score(pk.PK_POLICY_LEARNED))
    finally:
        pk.pk_case_table_set_learned_margin(t, 0.05)
    g_case, g_model, g_learned = geomean(case), geomean(model), geomean(learned)
    say("held-out %d shapes: CASE %.4f (worst %.3f), model alone %.4f (worst %.3f), LEARNED %.4f (worst %.3f)"
        % (len(shapes), g_case, min(case), g_model, min(model), g_learned, min(learned)))
    assert g_model > g_case
    assert g_learned >= g_model - 0.005
