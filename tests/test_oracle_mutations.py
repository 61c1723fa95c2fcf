"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a swapped weight, a wrong sign or index, a
dropped term) in a copy of the oracle's C source, builds it on the CPU, and
checks that at least one pin of ``test_oracle_pins`` fails against it, while
the unmodified source passes them all.  CPU only.
"""
import os

import pytest

from oracle import oracle as O
import test_oracle_pins as T


# Coherent alternative CG solvers: each converges to the same field as the
# paper's CG (so the converged pins pass), but its iterates before convergence
# differ.  They are whole-block replacements of the oracle's CG.
_CG_INIT = """    for (int32_t g = 0; g < ng; ++g) {
        phi[g] = 0.0;
        r[g] = g == 0 ? 0.0 : -rho[g] * dx * dx;
        d[g] = r[g];
    }"""
_CG_OP = """            for (int32_t g = 0; g < ng; ++g) {
                if (g == 0)
                    z[g] = d[0];
                else {
                    double right = g + 1 < ng ? d[g + 1] : 0.0;
                    z[g] = d[g - 1] - 2.0 * d[g] + right;
                }
            }"""
_CG_PIN_LAST_INIT = _CG_INIT.replace("r[g] = g == 0 ? 0.0", "r[g] = g == ng - 1 ? 0.0")
_CG_PIN_LAST_OP = """            for (int32_t g = 0; g < ng; ++g) {
                if (g == ng - 1)
                    z[g] = d[ng - 1];
                else {
                    double left = g > 0 ? d[g - 1] : 0.0;
                    z[g] = left - 2.0 * d[g] + d[g + 1];
                }
            }"""
_CG_JACOBI_START = """    for (int32_t g = 0; g < ng; ++g)
        phi[g] = g == 0 ? 0.0 : 0.5 * rho[g] * dx * dx;
    for (int32_t g = 0; g < ng; ++g) {
        double right = g + 1 < ng ? phi[g + 1] : 0.0;
        double aphi = g == 0 ? phi[0] : phi[g - 1] - 2.0 * phi[g] + right;
        r[g] = (g == 0 ? 0.0 : -rho[g] * dx * dx) - aphi;
        d[g] = r[g];
    }"""
_CG_LOOP = """    if (sqrt(rr) > 1e-16) {
        for (; it < maxit; ++it) {"""
_CG_CONJUGATE_RESIDUAL = """    if (sqrt(rr) > 1e-16) {
        double *ar = (double *)malloc(sz);
#define APPLY_A(out, in) for (int32_t g = 0; g < ng; ++g) { \\
            if (g == 0) out[g] = in[0]; \\
            else { double rt = g + 1 < ng ? in[g + 1] : 0.0; out[g] = in[g - 1] - 2.0 * in[g] + rt; } }
        APPLY_A(ar, r);
        for (int32_t g = 0; g < ng; ++g)
            z[g] = ar[g];
        double rar = 0.0;
        for (int32_t g = 0; g < ng; ++g)
            rar += r[g] * ar[g];
        for (; it < maxit; ++it) {
            double zz = 0.0;
            for (int32_t g = 0; g < ng; ++g)
                zz += z[g] * z[g];
            if (zz == 0.0)
                break;
            double alpha = rar / zz;
            for (int32_t g = 0; g < ng; ++g) {
                phi[g] += alpha * d[g];
                r[g] -= alpha * z[g];
            }
            APPLY_A(ar, r);
            double rar_new = 0.0;
            for (int32_t g = 0; g < ng; ++g)
                rar_new += r[g] * ar[g];
            double beta = rar_new / rar;
            for (int32_t g = 0; g < ng; ++g) {
                d[g] = r[g] + beta * d[g];
                z[g] = ar[g] + beta * z[g];
            }
            rar = rar_new;
        }
        free(ar);
    }
    if (0) {
        for (; it < maxit; ++it) {"""

# (name, original text, planted mistake); a mutant may also replace several
# texts at once (tuples of originals and of mistakes).
MUTANTS = [
    ("deposit weights swapped", "rho[j0] += (1.0 - f) * qdx;", "rho[j0] += f * qdx;"),
    ("node offset sign", "double t = x / cell_width(p) - 0.5;", "double t = x / cell_width(p) + 0.5;"),
    ("fixed half-cell shift sign", "int64_t Us = U - ((int64_t)1 << 31);", "int64_t Us = U + ((int64_t)1 << 31);"),
    ("fixed right node index", "S[wrap_index(j + 1, ng)] += F;", "S[wrap_index(j - 1, ng)] += F;"),
    ("fixed left weight", "S[wrap_index(j, ng)] += ((int64_t)1 << 32) - F;", "S[wrap_index(j, ng)] += F;"),
    ("solve drops mean", "run += (rho[g] - mean) * dx;", "run += rho[g] * dx;"),
    ("solve sign", "run += (rho[g] - mean) * dx;", "run -= (rho[g] - mean) * dx;"),
    ("solve neighbour index", "double left = face[g == 0 ? ng - 1 : g - 1];",
     "double left = face[g + 1 < ng ? g + 1 : 0];"),
    ("solve drops gauge constant", "face[g] -= c;", "face[g] -= 0.0 * c;"),
    ("kick sign", "double v_new = v_old + p->qm * Ep[i] * p->dt;", "double v_new = v_old - p->qm * Ep[i] * p->dt;"),
    ("drift with old velocity", "x[i] = wrap_position(p, x[i] + v_new * p->dt);",
     "x[i] = wrap_position(p, x[i] + v_old * p->dt);"),
    ("gather weights swapped", "Ep[i] = (1.0 - f) * E[j0] + f * E[j1];", "Ep[i] = f * E[j0] + (1.0 - f) * E[j1];"),
    ("field energy factor", "return 0.5 * s * cell_width(p);", "return s * cell_width(p);"),
    ("charge sign", "double s = p->qm < 0.0 ? -1.0 : 1.0;", "double s = p->qm < 0.0 ? 1.0 : -1.0;"),
    ("wrap with ceil", "x -= p->L * floor(x / p->L);", "x -= p->L * ceil(x / p->L);"),
    ("kinetic energy factor", "row[0] = 0.25 * m * (acc[0] + acc[1]);", "row[0] = 0.5 * m * (acc[0] + acc[1]);"),
    ("cg beta inverted", "double beta = rr_new / rr;", "double beta = rr / rr_new;"),
    ("cg pinned row", "r[g] = g == 0 ? 0.0 : -rho[g] * dx * dx;", "r[g] = -rho[g] * dx * dx;"),
    ("cell key half-cell shift sign", "double j = floor(u - 0.5);", "double j = floor(u + 0.5);"),
    ("cell order not stable", "for (int64_t i = 0; i < np; ++i)\n        perm[",
     "for (int64_t i = np - 1; i >= 0; --i)\n        perm["),
    ("literal cycle kicks with the wrong sign", "            v[i] = v[i] + p->qm * Ep[i] * p->dt;",
     "            v[i] = v[i] - p->qm * Ep[i] * p->dt;"),
    ("phase image transposed", "counts[row * nx + col] += 1;", "counts[col * nv + row] += 1;"),
    ("phase velocity offset sign", "double y = (w[i] - w_lo) * w_bin;", "double y = (w[i] + w_lo) * w_bin;"),
    ("phase column scale", "double xs = (double)nx / (double)p->ng;", "double xs = (double)nv / (double)p->ng;"),
    ("phase lower velocity edge excluded", "if (!(y >= 0.0 && y < (double)nv)) {",
     "if (!(y > 0.0 && y < (double)nv)) {"),
    ("cg pins the last node instead of node 0", (_CG_INIT, _CG_OP), (_CG_PIN_LAST_INIT, _CG_PIN_LAST_OP)),
    ("cg starts from the Jacobi guess", _CG_INIT, _CG_JACOBI_START),
    ("cg replaced by conjugate residual", _CG_LOOP, _CG_CONJUGATE_RESIDUAL),
]

# The pins run against every build (argument lists for the parametrised ones).
PINS = [
    (T.test_plain_deposit_matches_triangle_bruteforce, [(2,), (4,), (8,)]),
    (T.test_fixed_deposit_total_is_exact_and_matches_bruteforce, [(3,), (8,)]),
    (T.test_fixed_deposit_hand_derived_golden_cases, [()]),
    (T.test_phase_space_matches_bruteforce, [(8, 5), (3, 7)]),
    (T.test_phase_space_edges, [()]),
    (T.test_cell_order_hand_derived_case, [()]),
    (T.test_cell_order_is_a_stable_sort_by_nearest_node, [(5,), (64,)]),
    (T.test_fixed_density_matches_plain_density, [()]),
    (T.test_solve_matches_dense_linear_algebra, [(8,), (17,)]),
    (T.test_solve_single_mode_closed_form, [(16, 1), (64, 3)]),
    (T.test_paper_cg_converges_to_exact_solve, [(32,)]),
    (T.test_paper_cg_iterate_is_the_krylov_projection, [(64, 10), (256, 150)]),
    (T.test_gather_on_nodes_and_linear_field, [()]),
    (T.test_push_uniform_field_closed_form, [()]),
    (T.test_push_wraps_periodically, [()]),
    (T.test_momentum_is_conserved_to_rounding, [()]),
    (T.test_single_particle_feels_no_self_force, [(0.123,), (1.777,)]),
    (T.test_energy_conservation_two_stream, [()]),
    (T.test_cold_plasma_oscillates_at_the_discrete_plasma_frequency, [()]),
    (T.test_literal_cycle_order_equals_api_leapfrog_from_drifted_start, [()]),
    (T.test_warm_plasma_oscillates_at_the_bohm_gross_frequency, [()]),
]


def failing_pins():
    failed = []
    for fn, arglists in PINS:
        for args in arglists:
            try:
                fn(*args)
            except Exception as e:  # a crash of a broken build also counts as caught
                failed.append(f"{fn.__name__}{args}: {type(e).__name__}")
    return failed


@pytest.fixture
def restore_oracle():
    yield
    O.use_library(None)


def test_unmodified_oracle_passes_every_pin(restore_oracle):
    O.use_library(None)
    assert failing_pins() == []


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, orig, bad, tmp_path, restore_oracle):
    src = open(O.SRC).read()
    origs, bads = (orig, bad) if isinstance(orig, tuple) else ((orig,), (bad,))
    for o, b in zip(origs, bads):
        assert src.count(o) == 1, f"mutation anchor not unique: {o}"
        src = src.replace(o, b)
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src)
    so = O.build(str(mutant), str(tmp_path / f"libmutant_{abs(hash(name))}.so"))
    O.use_library(so)
    assert failing_pins(), f"no pin caught the planted mistake: {name}"
