"""Sensitivity of the oracle's pins: each plausible mistake below is planted in a copy of
oracle/oracle.c (on the CPU), the copy is compiled, and the oracle's own pin tests must fail
against it.  A mistake that every pin lets through would be an unpinned part of the oracle.

The planted mistakes cover every step the parity claims rest on: the congestion cost with its
history term (Eq. 3 marginal plus H), the DP's cost terms and tie rules (Alg. 3, Sec. III-D
look-ahead), the schedule's self-exclusion and history (negotiation rounds), the Elmore pass and
its reverse sweep (Sec. II-C, Fig. rc), Eq. 4/5 weights and the adjoint-form quantisation."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_dp.py", "tests/test_oracle_weights.py", "tests/test_oracle_elmore.py",
             "tests/test_oracle_quality.py", "tests/test_oracle_tree.py", "tests/test_oracle_batches.py",
             "tests/test_oracle_sta.py"]

TIE = "if (bl < 0 || key < bkey) { bl = lc; bkey = key; }"

# name -> (text in oracle.c, replacement, which occurrence: None = the only one)
MUTANTS = {
    # congestion cost: history term dropped or doubled; self-exclusion dropped; Eq. 3 s-value
    "kappa_history_dropped": ("+ (int64_t)H[g];", ";", None),
    "kappa_history_doubled": ("+ (int64_t)H[g];", "+ 2 * (int64_t)H[g];", None),
    "self_exclusion_dropped": ("(self_layer == l ? 1 : 0)", "0", None),
    "eq3_s_value": ("double s = z == 0 ? 0.5 : 1.5;", "double s = z == 0 ? 0.6 : 1.5;", None),
    # DP cost terms
    "via_range_shifted": ("for (int k = lo; k < hi; ++k) s += P->vr[k];",
                          "for (int k = lo + 1; k <= hi && k < P->L - 1; ++k) s += P->vr[k];", None),
    "pin_term_dropped": ("f += P->w_d * Tq(P->pin_w[T->sink_of[v]], rvia(P, l, 0), 2 * (int64_t)T->cpin[v]);",
                         ";", 0),
    "pi_model_half": ("Tq(P->seg_w[v], (int64_t)P->r[l] * T->len[v], Cs + 2 * Sn)",
                      "Tq(P->seg_w[v], (int64_t)P->r[l] * T->len[v], 2 * Cs + 2 * Sn)", None),
    "wire_weight_ignored": ("Tq(P->seg_w[v], (int64_t)P->r[l] * T->len[v], Cs + 2 * Sn)",
                            "Tq(1024, (int64_t)P->r[l] * T->len[v], Cs + 2 * Sn)", None),
    "lookahead_factor": ("fp = f + P->w_d * (((int64_t)P->lambda[v] * 2 * (Cs + Sn)) >> 11);",
                         "fp = f + P->w_d * (((int64_t)P->lambda[v] * (Cs + Sn)) >> 11);", None),
    "lookahead_sign": ("fp = f + P->w_d * (((int64_t)P->lambda[v] * 2 * (Cs + Sn)) >> 11);",
                       "fp = f - P->w_d * (((int64_t)P->lambda[v] * 2 * (Cs + Sn)) >> 11);", None),
    # tie rules: stacks (smallest b, then t) and a child's lowest layer, in either child loop
    "stack_tie_last": ("if (fp < best_fp)", "if (fp <= best_fp)", None),
    "child_tie_cost_loop": (TIE, TIE.replace("key < bkey", "key <= bkey"), 0),
    "child_tie_record_loop": (TIE, TIE.replace("key < bkey", "key <= bkey"), 1),
    # history saturation
    "history_unsaturated": ("H[g] = (int32_t)(h > HIST_SAT ? HIST_SAT : h);",
                            "H[g] = (int32_t)(h > 2 * HIST_SAT ? 2 * HIST_SAT : h);", None),
    # Elmore and its reverse sweep
    "elmore_half": ("t[v] = (p < 0 ? 0.0 : t[p]) + R[v] * (0.5 * C[v] + S[v]);",
                    "t[v] = (p < 0 ? 0.0 : t[p]) + R[v] * (C[v] + S[v]);", None),
    "adjoint_path_sum": ("Sig[v] = up + R[v] * G[v];", "Sig[v] = R[v] * G[v];", None),
    # Eq. 5 and the adjoint-form weights
    "eq5_self_sink": ("uint16_t w = T->is_sink[v] ? pin_w[T->sink_of[v]] : 0;", "uint16_t w = 0;", None),
    "adjoint_segw_scale": ("double q = nearbyint(-1024.0 * G[v]);", "double q = nearbyint(-1000.0 * G[v]);", None),
    "adjoint_pinw_scale": ("double q = nearbyint(-1024.0 * gbar[k]);", "double q = nearbyint(-1000.0 * gbar[k]);",
                           None),
    "adjoint_lambda_scale": ("nearbyint(-Sig[p] * 1e6)", "nearbyint(-Sig[p] * 1e3)", None),
    # classical batching: boxes that touch at one GCell, a box one GCell short, subsets sharing
    # batches
    "batch_touching_allowed": ("for (int32_t y = b[2]; y <= b[3] && free_here; ++y)",
                               "for (int32_t y = b[2] + 1; y <= b[3] && free_here; ++y)", None),
    "batch_box_short": ("if (T->x[v] > x1) x1 = T->x[v];", "if (T->x[v] > x1) x1 = T->x[v] - 1;", None),
    "batch_subsets_shared": ("base += nb;", "base += 0;", None),
    # static timing of the gate graph and Alg. 1's division
    "sta_gate_delay_dropped": ("AD[m] = (float)((double)gate_fs[m] * 1e-3) + in;", "AD[m] = in;", None),
    "sta_required_max": ("if (r < rd) rd = r;", "if (r > rd || rd == INFINITY) rd = r;", None),
    "sta_tie_last_input": ("if (best < 0 || AS[fin[j]] > AS[best]) best = fin[j];",
                           "if (best < 0 || AS[fin[j]] >= AS[best]) best = fin[j];", None),
    "sta_path_threshold": ("const float lim = 0.7f * wns;", "const float lim = 0.75f * wns;", None),
    "alg1_critical_from_three": ("        if (crit[n] > 3) {\n            int32_t k = 0;",
                                 "        if (crit[n] >= 3) {\n            int32_t k = 0;", None),
    "alg1_semi_threshold": ("if (wns < 0.0f && ns < 0.7f * wns) {", "if (wns < 0.0f && ns < 0.5f * wns) {", None),
}


def _mutate(src, old, new, which):
    n = src.count(old)
    if which is None:
        assert n == 1, (old, n)
        return src.replace(old, new)
    assert n > which, (old, n)
    pos = -1
    for _ in range(which + 1):
        pos = src.index(old, pos + 1)
    return src[:pos] + new + src[pos + len(old):]


def _caught(name, src, tmp):
    d = os.path.join(tmp, name)
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, "oracle.c")
    so = os.path.join(d, "liboracle.so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-o", so, c, "-lm"])
    env = dict(os.environ, GAPLA_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"] +
                       PIN_FILES, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode == 1


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        src = f.read()
    jobs = {name: _mutate(src, old, new, which) for name, (old, new, which) in MUTANTS.items()}
    with ThreadPoolExecutor(max_workers=4) as ex:
        res = dict(zip(jobs, ex.map(lambda kv: _caught(kv[0], kv[1], str(tmp_path)), jobs.items())))
    missed = [k for k, ok in res.items() if not ok]
    assert not missed, "mistakes no pin catches: %s" % missed


def test_unmutated_copy_passes_the_pins(tmp_path):
    # the harness itself: the oracle as committed, compiled the same way, passes every pin
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        src = f.read()
    assert not _caught("unmutated", src, str(tmp_path))
