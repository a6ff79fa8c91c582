"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
in a copy of an oracle source (a dropped term, a sign, an index, an
off-by-one, a constant): oracle/mc_oracle.c against the pins of
test_oracle_ising, test_oracle_join_update and test_oracle_rng_math;
oracle/mlp_oracle.c against those of test_oracle_mlp; oracle/thermo.py
against those of test_oracle_thermo.  The C copies are built with the
oracle's own flags and loaded in place of the oracle.  At least one pin must
fail.  Everything runs on the CPU, each case in a child process (the
oracle of the test run is never replaced).  A control case builds the
unchanged source the same way and must pass every pin."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
import oracle.build as OB  # noqa: E402

import test_oracle_ising as TI  # noqa: E402
import test_oracle_join_update as TJ  # noqa: E402
import test_oracle_mlp as TM  # noqa: E402
import test_oracle_rng_math as TR  # noqa: E402
import test_oracle_thermo as TT  # noqa: E402

# (name, text in mc_oracle.c, its replacement); each text occurs once
MUTANTS = [
    ("energy drops the down bond", "e -= (int64_t)s[j] * (s[right] + s[down]);", "e -= (int64_t)s[j] * s[right];"),
    ("flip energy has the wrong sign", "int dE = 2 * s[j] * h;", "int dE = -2 * s[j] * h;"),
    ("a neighbour counted twice", "int h = s[right] + s[left] + s[down] + s[up];",
     "int h = s[right] + s[left] + s[down] + s[down];"),
    ("acceptance compare reversed", "return u <= tau ? 1 : 0;", "return u >= tau ? 1 : 0;"),
    ("threshold difference transposed", "double d = lnW[mt >> bin_shift] - lnW[m >> bin_shift];",
     "double d = lnW[m >> bin_shift] - lnW[mt >> bin_shift];"),
    ("joint keeps from one past the accepted position",
     "for (int64_t k = kstar; k < M; ++k) H[", "for (int64_t k = kstar + 1; k < M; ++k) H["),
    ("seam taken from the first configuration", "sigma = tr[M - 1] + N / 2;", "sigma = tr[0] + N / 2;"),
    ("update adds ln h", "lnW[b] = lnW[b] - orc_log(H[b]);", "lnW[b] = lnW[b] + orc_log(H[b]);"),
    ("flatness ratio off", "5 * n * mn >= 4 * sum", "5 * n * mn >= 3 * sum"),
    ("Philox multiplier wrong", "M0 = 0xD2511F53u", "M0 = 0xD2511F55u"),
    ("initial spin from the wrong bit", "(orc_uniform(seed, L, 1u, 0u, c, (uint32_t)j) >> 31) ? 1 : -1",
     "(orc_uniform(seed, L, 1u, 0u, c, (uint32_t)j) & 1u) ? 1 : -1"),
    ("exp without the ln 2 tail", "r = fma(-k, orc_ln2_tail(), r);", "r = r + 0.0 * orc_ln2_tail();"),
    ("log series truncated", "for (int i = 10; i >= 1; --i) q = fma(q, z,",
     "for (int i = 6; i >= 1; --i) q = fma(q, z,"),
    ("threshold scaled by 2^32 - 1", "floor(orc_exp(d) * 4294967296.0)", "floor(orc_exp(d) * 4294967295.0)"),
]

# the pins, fastest first; a mutant usually fails one of the first few
PINS = [
    TR.test_threshold_closed_form,
    TI.test_tabulate_closed_form,
    TI.test_energy_single_flip_changes,
    TI.test_init_chain_bits,
    TI.test_lnW_zero_sweeps_are_deterministic,
    TI.test_tracked_level_matches_lattice,
    TJ.test_join_hand_built_cuts,
    TJ.test_join_lnW_zero_keeps_everything,
    TJ.test_update_closed_forms,
    TJ.test_flatness_integer_rule,
    TJ.test_blockwise_joint_equals_the_whole,
    TR.test_uniform_word_selection_and_keying,
    TR.test_det_exp_accuracy,
    TR.test_det_log_accuracy,
    TI.test_exact_multicanonical_weight_gives_flat_histogram,
    lambda: TI.test_boltzmann_weight_gives_canonical_ensemble(0.3),
    lambda: TI.test_reachable_levels_match_exact(4),
    TJ.test_join_acceptance_probability_is_metropolis,
    TI.test_energy_reproduces_kaufman_at_L4,
    TJ.test_recursion_converges_to_exact_dos_L4_levels,
    TR.test_uniform_is_uniform,
    TR.test_philox_matches_rocrand,
]


# the network oracle (mlp_oracle.c) and its pins
MLP_MUTANTS = [
    ("backward pass uses 1 - h for the tanh derivative", "d2[j] = dy * p[OFF_W3 + j] * (1.0 - h2[j] * h2[j]);",
     "d2[j] = dy * p[OFF_W3 + j] * (1.0 - h2[j]);"),
    ("first-layer gradient takes the other input", "grad[OFF_W1 + 2 * i] += d1[i] * xs[0];",
     "grad[OFF_W1 + 2 * i] += d1[i] * xs[1];"),
    ("output reads the first hidden layer", "for (int j = 0; j < H; ++j) o += p[OFF_W3 + j] * h2[j];",
     "for (int j = 0; j < H; ++j) o += p[OFF_W3 + j] * h1[j];"),
]
MLP_PINS = [TM.test_n_params, TM.test_forward_closed_forms, TM.test_gradient_against_central_differences]

# the reweighting oracle (thermo.py) and its pins
THERMO_MUTANTS = [
    ("specific heat misses a beta", "c = beta * beta * np.sum(p * (E - e_mean) ** 2)",
     "c = beta * np.sum(p * (E - e_mean) ** 2)"),
    ("free energy has the wrong sign", "f = -lnZ / beta", "f = lnZ / beta"),
    ("density of states not normalised", "lnD = lnD + (N * np.log(2.0) - _logsumexp(lnD))",
     "lnD = lnD + N * np.log(2.0)"),
    ("level energy offset", "E = (4 * m - 2 * N)", "E = (4 * m - N)"),
    ("unreachable levels counted", "return m[(m != 1) & (m != N - 1)]", "return m"),
]
THERMO_PINS = [TT.test_temperature_limits, TT.test_constant_shift_and_bins, TT.test_L4_against_every_configuration,
               TT.test_L8_against_kaufman]


def _mutated(tmp, name, old, new):
    src = open(os.path.join(ROOT, "oracle", name)).read()
    assert src.count(old) == 1, old
    path = os.path.join(tmp, name)
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    return path


def _build_mutant(tmp, old, new, name="mc_oracle.c"):
    srcs = {s: os.path.join(ROOT, "oracle", s) for s in ("mc_oracle.c", "mlp_oracle.c")}
    srcs[name] = _mutated(tmp, name, old, new)
    lib = os.path.join(tmp, "liboracle_mutant.so")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-o", lib,
           srcs["mc_oracle.c"], srcs["mlp_oracle.c"], "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return lib


def _first_failure(pins):
    for i, pin in enumerate(pins):
        try:
            pin()
        except Exception:  # an assertion, or an error the mistake causes
            return i
    return -1


def run_pins(lib, group="mc"):
    """Load `lib` in place of the oracle and run a group of pins; the index of
    the first pin that fails, or -1 when all pass (run in a child process, so
    that a mistake that crashes the C code cannot take the test run with it)."""
    OB.LIB = lib
    O._lib = None
    return _first_failure(PINS if group == "mc" else MLP_PINS)


def run_thermo_pins(path):
    """Run the reweighting pins with the functions of the source at `path`."""
    ns = {"__name__": "thermo_mutant"}
    exec(compile(open(path).read(), path, "exec"), ns)
    TT.thermo = ns["thermo"]
    return _first_failure(THERMO_PINS)


def _run_child(call):
    code = ("import sys; sys.path[:0] = [%r, %r]; import test_oracle_mutants as T; "
            "i = T.%s; print('first failing pin', i); sys.exit(0 if i >= 0 else 3)" % (ROOT, HERE, call))
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)


def _check_caught(p, name):
    # exit 0: a pin failed; killed by a signal: the mistake crashed a pin;
    # 3: every pin passed; anything else: the runner itself failed
    assert p.returncode != 3, "no pin fails with: " + name
    assert p.returncode == 0 or p.returncode < 0, p.stdout + p.stderr


def test_unchanged_sources_pass_every_pin(tmp_path):
    lib = _build_mutant(str(tmp_path), "int dE = 2 * s[j] * h;", "int dE = 2 * s[j] * h;")
    for call in ("run_pins(%r)" % lib, "run_pins(%r, 'mlp')" % lib,
                 "run_thermo_pins(%r)" % os.path.join(ROOT, "oracle", "thermo.py")):
        p = _run_child(call)
        assert p.returncode == 3, call + p.stdout + p.stderr


@pytest.mark.parametrize("name,old,new", MLP_MUTANTS, ids=[m[0] for m in MLP_MUTANTS])
def test_network_pins_catch_planted_mistake(name, old, new, tmp_path):
    lib = _build_mutant(str(tmp_path), old, new, "mlp_oracle.c")
    _check_caught(_run_child("run_pins(%r, 'mlp')" % lib), name)


@pytest.mark.parametrize("name,old,new", THERMO_MUTANTS, ids=[m[0] for m in THERMO_MUTANTS])
def test_reweighting_pins_catch_planted_mistake(name, old, new, tmp_path):
    path = _mutated(str(tmp_path), "thermo.py", old, new)
    _check_caught(_run_child("run_thermo_pins(%r)" % path), name)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, tmp_path):
    lib = _build_mutant(str(tmp_path), old, new)
    _check_caught(_run_child("run_pins(%r)" % lib), name)
