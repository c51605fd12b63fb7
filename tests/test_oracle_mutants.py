"""Each plausible mistake planted in a copy of the oracle's C source must be
caught by at least one pin.  The copies are built in a temporary directory
on the CPU; the real oracle is untouched."""
import os

import pytest

import oracle
import pins

# (name, original text, replacement): a dropped term, a wrong sign, a wrong
# or transposed index, a wrong scale, a mistake in a closed form.
MUTANTS = [
    ("rx_ignored", "Rb = 0.5 * (rt + rv);", "Rb = 0.5 * (rt + rt);"),
    ("full_path_not_half", "Rb = 0.5 * (rt + rv);", "Rb = (rt + rv);"),
    ("doppler_sign", "double phi = (psi_f + th_f) - ph_f;", "double phi = (psi_f + th_f) + ph_f;"),
    ("beat_sign", "double phi = (psi_f + th_f) - ph_f;", "double phi = (psi_f - th_f) - ph_f;"),
    ("channel_transposed", "int m = c / r->N, rr = c % r->N;", "int m = c % r->M, rr = c / r->M;"),
    ("beat_factor_two", "k->Kb = (2.0 * r->mu) / (r->c0 * r->Fs);", "k->Kb = (r->mu) / (r->c0 * r->Fs);"),
    ("carrier_dropped", "k->Kc = r->carrier_phase ? (2.0 * r->fc) / r->c0 : 0.0;", "k->Kc = 0.0;"),
    ("carrier_always", "k->Kc = r->carrier_phase ? (2.0 * r->fc) / r->c0 : 0.0;",
     "k->Kc = (2.0 * r->fc) / r->c0;"),
    ("doppler_no_Tb", "k->Kd = ((2.0 * r->fc) * r->Tb) / r->c0;", "k->Kd = (2.0 * r->fc) / r->c0;"),
    ("n_off_by_one", "term(psi, b, beta, a, n, l, &re, &im);", "term(psi, b, beta, a, n + 1, l, &re, &im);"),
    ("l_off_by_one", "term(psi, b, beta, a, n, l, &re, &im);", "term(psi, b, beta, a, n, l + 1, &re, &im);"),
    ("n_l_swapped_in_phase", "double th_f = frac(b * (double)n);", "double th_f = frac(b * (double)l);"),
    ("amp_squared", "*re = a * cos(ang);\n    *im = a * sin(ang);",
     "*re = a * a * cos(ang);\n    *im = a * a * sin(ang);"),
    ("conjugate_output", "o[2 * n + 1] += im;", "o[2 * n + 1] -= im;"),
    ("dz_uses_y", "double dz = (double)z - ant[2];", "double dz = (double)z - ant[1];"),
    ("dropped_dz", "return sqrt((dx * dx + dy * dy) + dz * dz);", "return sqrt(dx * dx + dy * dy);"),
    ("first_pixel_skipped", "for (int64_t p = 0; p < P; ++p) {", "for (int64_t p = 1; p < P; ++p) {"),
    ("entries_n_l_swapped", "strength(r, px, p, ls[k]), ns[k], ls[k], &re, &im);",
     "strength(r, px, p, ls[k]), ls[k] % r->Ns, ns[k] % r->L, &re, &im);"),
    ("marginal_l_sign", "geom(r->L, -beta, &gr, &gi);", "geom(r->L, beta, &gr, &gi);"),
    ("marginal_n_length", "geom(r->Ns, b, &gr, &gi);", "geom(r->Ns - 1, b, &gr, &gi);"),
    ("geom_phase_half", "double ang = PI * fmod((double)(N - 1) * xr, 2.0);",
     "double ang = PI * fmod((double)N * xr, 2.0);"),
    # signal-model variants
    ("slot_sign", "*psi = *psi - *beta * ((double)m / (double)r->M);",
     "*psi = *psi + *beta * ((double)m / (double)r->M);"),
    ("slot_whole_blocks", "*psi = *psi - *beta * ((double)m / (double)r->M);", "*psi = *psi - *beta * (double)m;"),
    ("slot_by_rx", "*psi = *psi - *beta * ((double)m / (double)r->M);",
     "*psi = *psi - *beta * ((double)rr / (double)r->M);"),
    ("intra_sign", "*b = *b - v * k->Kf;", "*b = *b + v * k->Kf;"),
    ("intra_uses_beat_constant", "*b = *b - v * k->Kf;", "*b = *b - v * k->Kb;"),
    ("rvp_sign", "*psi = *psi - (Rb * Rb) * k->Krvp;", "*psi = *psi + (Rb * Rb) * k->Krvp;"),
    ("rvp_factor", "k->Krvp = (2.0 * r->mu) / (r->c0 * r->c0);", "k->Krvp = (r->mu) / (r->c0 * r->c0);"),
    ("ff_beat_uses_expanded_range", "Rb = Rp;", "Rb = Rp - s;"),
    ("ff_no_half", "double s = 0.5 * ((ux", "double s = ((ux"),
    ("ff_sign", "ps = Rp * k->Kc - s * k->Ka;", "ps = Rp * k->Kc + s * k->Ka;"),
    ("ff_angle_scaled_by_carrier_switch", "ps = Rp * k->Kc - s * k->Ka;", "ps = (Rp - s) * k->Kc;"),
    ("ff_common_phase_always", "ps = Rp * k->Kc - s * k->Ka;", "ps = (Rp - s) * k->Ka;"),
    ("ff_angle_half_wavelength", "k->Ka = (2.0 * r->fc) / r->c0;", "k->Ka = r->fc / r->c0;"),
    ("block_strength_ignored", "if (r->model & ORC_BLOCK_STRENGTH) return", "if (0) return"),
    ("block_strength_transposed", "px->amp[(int64_t)l * px->P + p]", "px->amp[(int64_t)p * r->L + l]"),
    ("block_strength_next_block", "px->amp[(int64_t)l * px->P + p]",
     "px->amp[(int64_t)((l + 1) % r->L) * px->P + p]"),
    ("entries_block_of_row_zero", "term(psi, b, beta, strength(r, px, p, ls[k]),",
     "term(psi, b, beta, strength(r, px, p, 0),"),
    ("marginal_l_block_sign", "gi -= al * sin(th);", "gi += al * sin(th);"),
    ("ff_ignores_rx", "uz * (tx[2] + rx[2]));", "uz * (tx[2] + rx[2])) + 0.5 * ((ux * (tx[0] - rx[0]) + uy * (tx[1] - rx[1])) + uz * (tx[2] - rx[2]));"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = os.path.join(tmp_path, "mutant.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = oracle.build(src=path, out=os.path.join(tmp_path, "libmutant.so"))
    o = oracle.Oracle(lib)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(o)
        except (AssertionError, ValueError, FloatingPointError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
