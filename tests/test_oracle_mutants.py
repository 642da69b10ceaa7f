"""The pins catch plausible mistakes: each mutant below is the oracle's source
with one deliberate error (a flipped sign, a dropped term, a wrong constant
or operand), compiled on the CPU; the battery of pins of
test_oracle_pieces.py / test_oracle_scheme.py / test_oracle_fallback.py /
test_oracle_flatten.py / test_oracle_species.py is run against it and at least
one pin must fail.  Nothing here touches a GPU."""
import os
import subprocess
import tempfile

import pytest

import test_oracle_fallback as FB
import test_oracle_flatten as F
import test_oracle_pieces as P
import test_oracle_scheme as S
import test_oracle_species as SP

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hydro_oracle.c")

MUTANTS = {
    "corner correction sign": (
        "V[v] = Uq[v] - fac * (Fhi[v] - Flo[v]);",
        "V[v] = Uq[v] + fac * (Fhi[v] - Flo[v]);"),
    "final correction operand order": (
        "V[v] = (Uq[v] - f1 * (A1[v] - A0[v])) - f2 * (B1[v] - B0[v]);",
        "V[v] = (Uq[v] - f1 * (A0[v] - A1[v])) - f2 * (B1[v] - B0[v]);"),
    "dropped curvature term at the low face": (
        "return aL + (0.5 * s) * (dA + (1.0 - C23 * s) * a6);",
        "return aL + (0.5 * s) * dA;"),
    "tracing velocity sign": (
        "f[1] = r_un + cor * am;",
        "f[1] = r_un - cor * am;"),
    "HLLC right wave speed min for max": (
        "double SR = mx(uL + cL, uR + cR);",
        "double SR = mn(uL + cL, uR + cR);"),
    "reflect without momentum flip": (
        "U[c * cs + dst] = (hydro && flip && c == 1 + d) ? -v : v;",
        "U[c * cs + dst] = v;"),
    "z flux divergence sign": (
        "du = du + dtdx[2] * (fat(&F3[2], pz)[v] - fat(&F3[2], p)[v]);",
        "du = du - dtdx[2] * (fat(&F3[2], pz)[v] - fat(&F3[2], p)[v]);"),
    "gravity energy source term": (
        "Us[4] = Us[4] + hg * (Un[1 + e] + mnew);",
        "Us[4] = Us[4] + hg * (Un[1 + e] + Un[1 + e]);"),
    "interface value constant": (
        "double aL = 0.5 * (a[1] + a[2]) - (d0 - dm) * C6;",
        "double aL = 0.5 * (a[1] + a[2]) - (d0 - dm) * C23;"),
    "CFL number dropped": (
        "*dt = pr->cfl * mn(",
        "*dt = 1.0 * mn("),
    "minmod-like slope bound": (
        "return copysign(mn(mn(fabs(dc), 2.0 * fabs(dl)), 2.0 * fabs(dr)), dc);",
        "return copysign(mn(mn(fabs(dc), fabs(dl)), 2.0 * fabs(dr)), dc);"),
    "HLLC star energy pressure-work sign": (
        "Us[4] = chi * (E + (rho * (Ss - uK)) * (Ss + pK / (rho * (SK - uK))));",
        "Us[4] = chi * (E + (rho * (Ss - uK)) * (Ss - pK / (rho * (SK - uK))));"),
    "HLLC star normal momentum": (
        "Us[1 + d] = chi * (rho * Ss);",
        "Us[1 + d] = chi * (rho * uK);"),
    "entropy wave amplitude sign": (
        "double az = lam[1] > 0.0 ? drz - dpz * ics2 : 0.0;",
        "double az = lam[1] > 0.0 ? drz + dpz * ics2 : 0.0;"),
    "corner coupling factor dt/2 for dt/3": (
        "goto done; }\n            const double fac = dt / (3.0 * b->dx[sd]);",
        "goto done; }\n            const double fac = dt / (2.0 * b->dx[sd]);"),
    "flattening reaches toward the higher pressure": (
        "int s = p7[4] > p7[2] ? -1 : 1;",
        "int s = p7[4] > p7[2] ? 1 : -1;"),
    "flattening without the compression test": (
        "int shock = (u3[0] - u3[2] > 0.0) && (fabs(dp) > FL_EPS * mn(p5[3], p5[1]));",
        "int shock = fabs(dp) > FL_EPS * mn(p5[3], p5[1]);"),
    "flattening weights swapped": (
        "aL = f * aL + (1.0 - f) * ac;",
        "aL = (1.0 - f) * aL + f * ac;"),
    "species donor side swapped": (
        "fat(&G1[d], p)[sp] = F * (F >= 0.0 ? fat(&Xhi[d], l)[sp] : fat(&Xlo[d], p)[sp]);",
        "fat(&G1[d], p)[sp] = F * (F >= 0.0 ? fat(&Xlo[d], p)[sp] : fat(&Xhi[d], l)[sp]);"),
    "species traced on the fast wave": (
        "un > 0.0 ? un : un + c",
        "un + c"),
    "species corner correction sign": (
        "rq * xq[sp] - fac * (fat(&G1[sd], cu)[sp] - fat(&G1[sd], c)[sp]);",
        "rq * xq[sp] + fac * (fat(&G1[sd], cu)[sp] - fat(&G1[sd], c)[sp]);"),
    "species final correction operand": (
        "f2 * (fat(&G2[t2][t1], c2)[sp] - fat(&G2[t2][t1], c)[sp]);",
        "f2 * (fat(&G2[t2][t1], c1)[sp] - fat(&G2[t2][t1], c)[sp]);"),
    "species update y-difference sign": (
        "du = du + dtdx[1] * (fat(&G3[1], py)[sp] - fat(&G3[1], p)[sp]);",
        "du = du - dtdx[1] * (fat(&G3[1], py)[sp] - fat(&G3[1], p)[sp]);"),
    "fallback rejects only negative density": (
        "if (rho <= 0.0 || p <= 0.0) {",
        "if (rho < 0.0 || p <= 0.0) {"),
    "fallback tests the pressure only": (
        "if (rho <= 0.0 || p <= 0.0) {",
        "if (p <= 0.0) {"),
    "fallback flag dropped": (
        "return ORC_ERR_FALLBACK;",
        "return 0;"),
    "corner fallback keeps the corrected state": (
        "err |= accept_state(V, q, gm1, qc[side]);",
        "err |= accept_state(V, V, gm1, qc[side]);"),
    "update pressure bit dropped": (
        "if (qn[4] <= 0.0) err |= ORC_ERR_P;",
        ""),
    "update density bit strict": (
        "if (Us[0] <= 0.0) err |= ORC_ERR_RHO;",
        "if (Us[0] < 0.0) err |= ORC_ERR_RHO;"),
    "species corner density reset dropped": (
        "xc[side][sp] = den > 0.0 ? num / den : xq[sp];",
        "xc[side][sp] = num / den;"),
    "species final density reset dropped": (
        "xf[side][sp] = den > 0.0 ? num / den : xq[sp];",
        "xf[side][sp] = num / den;"),
    "flattening steepness threshold": (
        "double chi = mn(1.0, mx(0.0, FL_W2 * (z - FL_W1)));",
        "double chi = mn(1.0, mx(0.0, FL_W2 * (z - 0.5)));"),
}

# the pins, cheapest first; each raises AssertionError when it fails
BATTERY = [
    ("fill vs numpy.pad", lambda o: S.test_fill_ghosts_matches_numpy_pad(o, ((2, 1, 0), (2, 1, 0)))),
    ("dt closed form", lambda o: S.test_dt_closed_form_sod(o)),
    ("PPM cubic", lambda o: P.test_ppm_interfaces_exact_on_cubic(o)),
    ("PPM monotone", lambda o: P.test_ppm_limited_parabola_monotone_and_conservative(o)),
    ("PPM quadrature", lambda o: P.test_ppm_integral_matches_quadrature(o)),
    ("trace entropy wave", lambda o: (P.test_trace_entropy_wave_is_upwind_average(o, 0.7),
                                      P.test_trace_entropy_wave_is_upwind_average(o, -0.7))),
    ("HLLC consistency", lambda o: P.test_hllc_consistency(o)),
    ("HLLC mirror", lambda o: P.test_hllc_mirror_symmetry(o)),
    ("HLLC contact", lambda o: (P.test_hllc_stationary_contact(o), P.test_hllc_moving_contact_is_upwind(o))),
    ("corrected-state rule", lambda o: ([FB.test_rejected_state_keeps_the_uncorrected_one(o, v, w)
                                         for v, w in FB.REJECTED],
                                        FB.test_accepted_state_is_its_primitive_form(o))),
    ("update bits closed form", lambda o: [FB.test_update_error_bits_on_expansion_closed_form(o, 1, s, b)
                                           for s, b in FB.EXPANSION_CASES]),
    ("non-finite reach", lambda o: FB.test_nonfinite_input_raises_bit_1_within_the_stencil_reach(o)),
    ("uniform state", lambda o: S.test_uniform_state_preserved_bitwise(o)),
    ("free fall", lambda o: S.test_free_fall_gravity_closed_form(o)),
    ("Sod permutation", lambda o: S.test_sod_axis_permutation_bitwise(o, 2)),
    ("Sod mirror", lambda o: S.test_sod_mirror_symmetry(o)),
    ("conservation", lambda o: S.test_conservation_periodic(o, "kh")),
    ("walls conserve", lambda o: S.test_reflecting_walls_conserve_mass_energy(o)),
    ("CTU stability", lambda o: S.test_ctu_stable_near_unit_courant_number(o)),
    ("sound waves in streams", lambda o: [S.test_sound_wave_in_stream_second_order(o, u, s)
                                          for u, s in [(2.0, 1), (2.0, -1), (-2.0, 1),
                                                       (-2.0, -1), (0.3, 1)]]),
    ("Sod exact", lambda o: S.test_sod_against_exact_solution(o)),
    ("smooth order 2-D", lambda o: S.test_smooth_advection_second_order_2d(o)),
    ("smooth order 3-D", lambda o: S.test_smooth_advection_second_order_3d(o)),
    ("flattening coefficient", lambda o: F.test_coefficient_worked_examples(o)),
    ("flattening toward the mean", lambda o: F.test_flattening_limits_the_parabola_toward_the_mean(o)),
    ("full flattening first order", lambda o: F.test_full_flattening_is_first_order(o)),
    ("strong shock marked", lambda o: F.test_coefficient_marks_a_strong_shock_only(o)),
    ("first-order CTU", lambda o: [FB.test_first_step_on_piecewise_constant_data_is_first_order_ctu(o, *c)
                                   for c in FB.CTU_CASES]),
    ("species unit fraction", lambda o: [SP.test_unit_fraction_is_the_density_bitwise(o, c)
                                         for c in ("kh", "rt")]),
    ("species 1-D advection", lambda o: [SP.test_uniform_flow_is_1d_ppm_advection(o, a, u)
                                         for a in (0, 1, 2) for u in (0.6, -1.7)]),
    ("species CTU advection", lambda o: [SP.test_oblique_uniform_flow_is_ctu_advection(o, v)
                                         for v in ((0.7, -0.5, 0.4), (-1.6, 0.3, -0.9))]),
]


def _build_mutant(name, tmp):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found (or not unique): %s" % name
    path = os.path.join(tmp, "hydro_oracle.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    hdr = os.path.join(ROOT, "oracle", "hydro_oracle.h")
    lib = os.path.join(tmp, "libmutant.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11", "-shared", "-fPIC",
                    "-w", "-I", os.path.dirname(hdr), "-o", lib, path, "-lm"], check=True)
    return lib


def _first_failing_pin(orc):
    for label, check in BATTERY:
        try:
            check(orc)
        except AssertionError:
            return label
        except (ValueError, MemoryError, FloatingPointError):
            return label + " (error)"
    return None


def test_unmutated_oracle_passes_battery(orc):
    assert _first_failing_pin(orc) is None


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(orc, name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(name, tmp)
        with orc.using(lib):
            caught = _first_failing_pin(orc)
    print("%s: caught by %s" % (name, caught))
    assert caught is not None, "no pin fails for the mutant '%s'" % name
