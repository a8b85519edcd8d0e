"""Opt-in: plausible mistakes planted anywhere in the oracle's arithmetic each make a CPU pin
fail.

Each case plants one mistake (a dropped term, a wrong sign, factor or index, a transposed
operand, a step taken at the wrong point) in a copy of qcqp_oracle.c, builds the copy with the
oracle's own flags and runs every oracle pin (tests/test_oracle_*.py without the sanitizer run)
against it in a child process (ORACLE_LIB names the copy); the run must report a failure.  The
cases cover the operator and its storage decoders, the stored-matrix map, the constraint values
and gradient, the dual-domain projections (orthant, simplex, second-order cones, balls, and
their order), both test functions and their steps, the averages, the step-size rule and its
state shift, the relative KKT residual (orthant, simplex and cone forms), the §5.1 criterion,
G_xi, the epoch start (momentum reset) and the restart point's evaluation.  The restart
driver's cases run by default in tests/test_restart_pins_catch_mistakes.py.

One measured mistake is left out because it changes no result: dropping the gradient restart of
the box-QP inner loop of G_xi only slows that loop, which still converges to the same minimiser.

The whole set takes several minutes, so it runs only with ORACLE_MUTANTS=1 in the environment.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "qcqp_oracle.c")

MISTAKES = {
    'Ax_minus_b_sign': (
        'for (int64_t l = 0; l < p; ++l) Gy[l] = dot(P->A + l * n, x, n) - P->b[l];',
        'for (int64_t l = 0; l < p; ++l) Gy[l] = dot(P->A + l * n, x, n) + P->b[l];'),
    'avg_from_y_old': (
        '    for (int64_t l = 0; l < ny; ++l) S->cy[l] += tk * S->yt[l];',
        '    for (int64_t l = 0; l < ny; ++l) S->cy[l] += tk * S->y[l];'),
    'avg_weight_uniform': (
        'double tk = sig / ep->sig0;',
        'double tk = 1.0;'),
    'ball_before_cone': (
        '    project_kstar(P, lam);\n    if (P->ball > 0.0) scale_to_ball(y, p + m, P->ball);',
        '    if (P->ball > 0.0) scale_to_ball(y, p + m, P->ball);\n    project_kstar(P, lam);'),
    'ball_not_applied': (
        '    if (P->ball > 0.0) scale_to_ball(y, p + m, P->ball);',
        '    if (P->ball > 1e300) scale_to_ball(y, p + m, P->ball);'),
    'cone_kkt_infeas_not_projected': (
        '        project_kstar(P, w);\n        project_kstar(P, gv);',
        '        project_kstar(P, w);'),
    'cone_maxv_block': (
        '            double b = sqrt(nrm2sq(gv + off, P->soc_dims[c]));\n            if (b > maxv) maxv = b;',
        '            double b = gv[off];\n            if (b > maxv) maxv = b;'),
    'epoch_alpha_tau': (
        'ep->alpha_k = (o->variant == 0) ? o->c_alpha / ep->sig_prev : o->c_alpha / ep->tau_prev;',
        'ep->alpha_k = (o->variant == 0) ? o->c_alpha / ep->tau_prev : o->c_alpha / ep->tau_prev;'),
    'epoch_keeps_momentum_x': (
        '    memcpy(S->Gyp, S->Gy, sizeof(double) * S->ny);\n    memcpy(S->gxp, S->gxk, sizeof(double) * S->n);\n    memset(S->cx',
        '    memcpy(S->Gyp, S->Gy, sizeof(double) * S->ny);\n    memset(S->cx'),
    'epoch_keeps_momentum_y': (
        '    memcpy(S->Gyp, S->Gy, sizeof(double) * S->ny);\n    memcpy(S->gxp, S->gxk, sizeof(double) * S->n);\n    memset(S->cx',
        '    memcpy(S->gxp, S->gxk, sizeof(double) * S->n);\n    memset(S->cx'),
    'eta_not_applied_once': (
        '        ep->tau *= o->eta;                   /* tau_k <- eta tau_k */',
        '        ep->tau *= o->eta * o->eta;'),
    'f16_bias': (
        'else v = ldexp((double)(mant + 1024), e - 25);',
        'else v = ldexp((double)(mant + 1024), e - 24);'),
    'f16_subnormal_exp': (
        'if (e == 0) v = ldexp((double)mant, -24);',
        'if (e == 0) v = ldexp((double)mant, -25);'),
    'g_half_dropped': (
        'double gi = 0.5 * dot(x, U + i * n, n) + dot(P->q + i * n, x, n) + P->c[i];',
        'double gi = dot(x, U + i * n, n) + dot(P->q + i * n, x, n) + P->c[i];'),
    'g_no_c': (
        'double gi = 0.5 * dot(x, U + i * n, n) + dot(P->q + i * n, x, n) + P->c[i];',
        'double gi = 0.5 * dot(x, U + i * n, n) + dot(P->q + i * n, x, n);'),
    'gamma_growth_sigma': (
        'double gam_next = ep->gam * (1.0 + o->mu * tau);',
        'double gam_next = ep->gam * (1.0 + o->mu * sig);'),
    'gap_H_no_q0': (
        '            double h = sidx[0] >= 0 ? qel(P, sidx[0], r, j) : 0.0;',
        '            double h = 0.0;'),
    'gap_H_no_shift': (
        'H[r * n + j] = h + (r == j ? 2.0 * xi + P->q0_shift : 0.0);',
        'H[r * n + j] = h + (r == j ? 2.0 * xi : 0.0);'),
    'gap_H_xi_not_2xi': (
        'H[r * n + j] = h + (r == j ? 2.0 * xi + P->q0_shift : 0.0);',
        'H[r * n + j] = h + (r == j ? xi + P->q0_shift : 0.0);'),
    'gap_Py_2xi': (
        'for (int64_t l = 0; l < p + m; ++l) yp[l] = y[l] + Gy[l] / (2.0 * xi);',
        'for (int64_t l = 0; l < p + m; ++l) yp[l] = y[l] + Gy[l] / xi;'),
    'gap_Py_sign': (
        '            Py += Gy[l] * dl - xi * dl * dl;',
        '            Py += Gy[l] * dl + xi * dl * dl;'),
    'gap_clip_box_absolute': (
        '            Dn[r] = clip(Z[r] - gz[r] / L, P->lb[r] - x[r], P->ub[r] - x[r]);',
        '            Dn[r] = clip(Z[r] - gz[r] / L, P->lb[r], P->ub[r]);'),
    'gap_hv_half_dropped': (
        'hv += gx[r] * D[r] + 0.5 * D[r] * dot(H + r * n, D, n);',
        'hv += gx[r] * D[r] + D[r] * dot(H + r * n, D, n);'),
    'grad_no_Atv': (
        '        for (int64_t j = 0; j < n; ++j) gx[j] += y[l] * P->A[l * n + j];\n}',
        '        for (int64_t j = 0; j < n; ++j) gx[j] += 0.0 * y[l] * P->A[l * n + j];\n}'),
    'grad_no_qi': (
        'for (int64_t j = 0; j < n; ++j) gx[j] += lam * (U[i * n + j] + P->q[i * n + j]);',
        'for (int64_t j = 0; j < n; ++j) gx[j] += lam * U[i * n + j];'),
    'kkt_comp_min_sign': (
        'double mn = lam < -g ? lam : -g;',
        'double mn = lam < g ? lam : g;'),
    'kkt_comp_norm_with_b': (
        '    double rel_comp = sqrt(rl) / (1.0 + sqrt(cn));',
        '    double rel_comp = sqrt(rl) / (1.0 + sqrt(cn) + sqrt(bn));'),
    'kkt_dual_denominator_s1': (
        'double rel_dual = sqrt(rx) / (1.0 + sqrt(s0) + sqrt(s1) + sqrt(s2));',
        'double rel_dual = sqrt(rx) / (1.0 + sqrt(s0) + sqrt(s2));'),
    'kkt_pri_includes_negative_g': (
        '            if (g > 0) { pri += g * g; if (g > maxv) maxv = g; }',
        '            { pri += g * g; if (g > maxv) maxv = g; }'),
    'kkt_pri_no_b': (
        '    double rel_pri = sqrt(pri) / (1.0 + sqrt(cn) + sqrt(bn));',
        '    double rel_pri = sqrt(pri) / (1.0 + sqrt(cn));'),
    'kkt_rx_sign': (
        'double r = x[j] - clip(x[j] - gj, P->lb[j], P->ub[j]);',
        'double r = x[j] - clip(x[j] + gj, P->lb[j], P->ub[j]);'),
    'kstar_no_clip': (
        '        if (lam[i] < 0.0) lam[i] = 0.0;',
        '        if (lam[i] < -1e300) lam[i] = 0.0;'),
    'matvec_no_shift': (
        'if (i == 0) s += P->q0_shift * x[r];',
        'if (0) s += P->q0_shift * x[r];'),
    'matvec_transposed': (
        'for (int64_t j = 0; j < n; ++j) s += qel(P, si, r, j) * x[j];',
        'for (int64_t j = 0; j < n; ++j) s += qel(P, si, j, r) * x[j];'),
    'no_q0_index': (
        '    if (!P->has_q0) return i == 0 ? -1 : i - 1;',
        '    if (!P->has_q0) return i == 0 ? -1 : i;'),
    'nonmono_one_dropped': (
        'double tau_next = tau * sqrt(ep->gam / gam_next * (1.0 + o->c_nm * tau / ep->tau_prev));',
        'double tau_next = tau * sqrt(ep->gam / gam_next * (o->c_nm * tau / ep->tau_prev));'),
    'paper_eq_not_abs': (
        '    for (int64_t l = 0; l < p; ++l) viol += fabs(Gy[l]);',
        '    for (int64_t l = 0; l < p; ++l) viol += Gy[l];'),
    'paper_mean_over_m': (
        'double mv = cnt > 0 ? viol / (double)cnt : 0.0;',
        'double mv = m > 0 ? viol / (double)m : 0.0;'),
    'restart_point_not_installed': (
        '        for (int64_t l = 0; l < S->ny; ++l) S->y[l] = S->cy[l] / S->T;\n        install_point(S);',
        '        for (int64_t l = 0; l < S->ny; ++l) S->y[l] = S->cy[l] / S->T;'),
    'rhs_delta_dual_dropped': (
        'rhs = -(o->delta / tau) * Dp - (o->delta / sig) * Dd;\n            if (E <= rhs) {\n                ep->alpha_k = alpha_next;\n                break;',
        'rhs = -(o->delta / tau) * Dp;\n            if (E <= rhs) {\n                ep->alpha_k = alpha_next;\n                break;'),
    'separable_ball_l_skipped': (
        '    if (P->ball_l > 0.0) scale_to_ball(lam, m, P->ball_l);',
        '    if (P->ball_l > 1e300) scale_to_ball(lam, m, P->ball_l);'),
    'separable_ball_v_on_all': (
        '    if (P->ball_v > 0.0) scale_to_ball(y, p, P->ball_v);',
        '    if (P->ball_v > 0.0) scale_to_ball(y, p + m, P->ball_v);'),
    'sigma_prev_not_shifted': (
        '    ep->sig_prev = sig;\n    ep->tau_prev = tau;',
        '    ep->tau_prev = tau;'),
    'simplex_kkt_sign': (
        '        for (int64_t i = 0; i < m; ++i) w[i] = y[p + i] + Gy[p + i];\n        project_simplex(w, m);',
        '        for (int64_t i = 0; i < m; ++i) w[i] = y[p + i] - Gy[p + i];\n        project_simplex(w, m);'),
    'simplex_no_clip': (
        '    for (int64_t i = 0; i < k; ++i) z[i] = z[i] > theta ? z[i] - theta : 0.0;',
        '    for (int64_t i = 0; i < k; ++i) z[i] = z[i] - theta;'),
    'simplex_theta_last': (
        '        if (u[j] > t) theta = t;',
        '        theta = t;'),
    'soc_no_half': (
        '    double a = 0.5 * (t + un);',
        '    double a = (t + un);'),
    'soc_polar_not_zeroed': (
        '    if (un <= -t) {\n        for (int64_t i = 0; i < k; ++i) z[i] = 0.0;\n        return;\n    }',
        '    if (un <= -t - 1e300) {\n        for (int64_t i = 0; i < k; ++i) z[i] = 0.0;\n        return;\n    }'),
    'soc_scale_wrong': (
        '    for (int64_t i = 1; i < k; ++i) z[i] *= a / un;',
        '    for (int64_t i = 1; i < k; ++i) z[i] *= a / (un + t);'),
    'stored_index_skip': (
        '        for (int64_t k = 0; k < i; ++k) s += P->q_stored[k] ? 1 : 0;',
        '        for (int64_t k = 0; k < i; ++k) s += 1;'),
    'theta_inverted': (
        '        th = ep->sig_prev / sig;             /* theta_k = sigma_{k-1} / sigma_k */',
        '        th = sig / ep->sig_prev;'),
    'trace_tau_next': (
        '        trace_row[0] = tau; trace_row[1] = sig;',
        '        trace_row[0] = tau_next; trace_row[1] = sig;'),
    'xy_E_Dd_sign': (
        '            E = nrm2sq(S->gtmp, n) / (2.0 * alpha_next) - Dd / sig +',
        '            E = nrm2sq(S->gtmp, n) / (2.0 * alpha_next) + Dd / sig +'),
    'xy_E_no_beta_term': (
        'nrm2sq(S->gtmp2, n) / (2.0 * beta_next) -',
        '0.0 * nrm2sq(S->gtmp2, n) / (2.0 * beta_next) -'),
    'xy_alpha_sig': (
        'double alpha_next = o->c_alpha / tau;',
        'double alpha_next = o->c_alpha / sig;'),
    'xy_beta_gamma0_dropped': (
        'double beta_next = o->gamma0 * o->c_beta / sig;',
        'double beta_next = o->c_beta / sig;'),
    'xy_dual_uses_old_G': (
        'for (int64_t l = 0; l < ny; ++l) S->yt[l] = S->y[l] + sig * S->Gyt[l];',
        'for (int64_t l = 0; l < ny; ++l) S->yt[l] = S->y[l] + sig * S->Gy[l];'),
    'xy_gtmp_no_A': (
        '                for (int64_t l = 0; l < p; ++l) a += (S->yt[l] - S->y[l]) * P->A[l * n + j];',
        '                for (int64_t l = 0; l < p; ++l) a += 0.0 * (S->yt[l] - S->y[l]) * P->A[l * n + j];'),
    'xy_no_momentum': (
        'S->s[j] = (1.0 + th) * S->gxk[j] - th * S->gxp[j];',
        'S->s[j] = S->gxk[j];'),
    'yx_E_no_dG': (
        'E = quad - Dp / tau + dG / (2.0 * alpha_next) - (1.0 / sig - th * ep->alpha_k) * Dd;',
        'E = quad - Dp / tau - (1.0 / sig - th * ep->alpha_k) * Dd;'),
    'yx_E_quad_sign': (
        'E = quad - Dp / tau + dG / (2.0 * alpha_next) - (1.0 / sig - th * ep->alpha_k) * Dd;',
        'E = -quad - Dp / tau + dG / (2.0 * alpha_next) - (1.0 / sig - th * ep->alpha_k) * Dd;'),
    'yx_E_theta_alpha_dropped': (
        'E = quad - Dp / tau + dG / (2.0 * alpha_next) - (1.0 / sig - th * ep->alpha_k) * Dd;',
        'E = quad - Dp / tau + dG / (2.0 * alpha_next) - (1.0 / sig) * Dd;'),
    'yx_alpha_next_tau': (
        'double alpha_next = o->c_alpha / sig;                    /* alpha_{k+1} = c_a / sigma_k */',
        'double alpha_next = o->c_alpha / tau;'),
    'yx_grad_at_old_y': (
        '            grad_x(P, S->U, S->yt, S->gtmp);',
        '            grad_x(P, S->U, S->y, S->gtmp);'),
    'yx_no_momentum': (
        'S->s[l] = (1.0 + th) * S->Gy[l] - th * S->Gyp[l];',
        'S->s[l] = S->Gy[l];'),
    'yx_quad_no_lambda': (
        '                double w = (i == 0) ? 1.0 : S->yt[p + i - 1];',
        '                double w = 1.0;'),
    'yx_quad_old_lambda': (
        '                double w = (i == 0) ? 1.0 : S->yt[p + i - 1];',
        '                double w = (i == 0) ? 1.0 : S->y[p + i - 1];'),
}


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("ORACLE_MUTANTS") != "1", reason="opt-in: set ORACLE_MUTANTS=1")
@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_oracle_pins_fail_on_planted_mistake(name, tmp_path):
    from oracle import build
    src = open(SRC).read()
    old, new = MISTAKES[name]
    assert src.count(old) == 1, f"the text the mistake replaces is no longer in qcqp_oracle.c: {old!r}"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = build.build_from(str(path), str(tmp_path / f"lib_{name}.so"))
    pins = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                  if f.startswith("test_oracle_") and f.endswith(".py") and f != "test_oracle_sanitized.py")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *pins], cwd=ROOT, env=dict(os.environ, ORACLE_LIB=lib), capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 1 and " failed" in r.stdout, tail
