"""Planted mistakes in the oracle (CPU only): each mutant copy of the oracle
source, compiled on its own, must fail at least one pin.  This shows the pins
would catch a dropped term, a wrong index or a transposed operand."""
import ctypes
import subprocess
from pathlib import Path

import pytest

import oracle
import oracle_pins as P

SRC = Path(oracle.__file__).resolve().parent / "fw_oracle.c"

MUTANTS = {
    "pick_ge": ("if (prefix > r) return", "if (prefix >= r) return"),
    "swap_return_out": ("f = p->f_ret;", "f = p->f_out;"),
    "drop_in_factor": ("f = p->f_in;", "f = 1;"),
    "schema_index": ("p->schema[t % p->schema_len]", "p->schema[(t + 1) % p->schema_len]"),
    "first_hop_rule": ("if (algo == FWO_NODE2VEC && t > 0) {", "if (algo == FWO_NODE2VEC && t > 1) {"),
    "draw_operands": ("fwo_draw(seed, qid, t)", "fwo_draw(seed, t, qid)"),
    "philox_key_bump": ("k1 += PHILOX_W1;", "k1 += 0;"),
    "philox_rounds": ("round < 10", "round < 9"),
    "scale_bias": ("(unsigned __int128)u * total", "(unsigned __int128)(u >> 1) * total"),
    "drop_weight": ("w_out[i] = w * f;", "w_out[i] = f;"),
    "ppr_coin_word": ("return fwo_stop_coin(out[1], stop_num, stop_den);",
                      "return fwo_stop_coin(out[0], stop_num, stop_den);"),
    "ppr_coin_le": ("(uint64_t)(p >> 64) < stop_num;", "(uint64_t)(p >> 64) <= stop_num;"),
    "ppr_coin_hop": ("fwo_stop(seed, qid, t, p->stop_num", "fwo_stop(seed, qid, t + 1, p->stop_num"),
    "ppr_first_coin": ("if (algo == FWO_PPR && fwo_stop(", "if (algo == FWO_PPR && t > 0 && fwo_stop("),
    "entry_word": ("return out[i % 4];", "return out[(i + 1) % 4];"),
    "entry_counter": ("uint64_t ctr[4] = {qid, t, i / 4, 1};", "uint64_t ctr[4] = {qid, t, i / 4, 0};"),
    "zigzag_partial_quad": ("uint64_t quads = (d + 3) / 4, m = 0;", "uint64_t quads = d / 4, m = 0;"),
    "reservoir_le": ("if ((uint64_t)(p >> 64) < w[i]) selected", "if ((uint64_t)(p >> 64) <= w[i]) selected"),
    "reservoir_exclusive_total": (
        "    total += w[i];\n    unsigned __int128 p = (unsigned __int128)u[i] * total;\n"
        "    if ((uint64_t)(p >> 64) < w[i]) selected = (int64_t)i;",
        "    unsigned __int128 p = (unsigned __int128)u[i] * total;\n"
        "    if ((uint64_t)(p >> 64) < w[i]) selected = (int64_t)i;\n    total += w[i];"),
    "alias_fill": ("rem -= T - q;", "rem -= T - q - 1;"),
    "alias_heavy_prob": ("prob[j] = rem;", "prob[j] = T;"),
    "alias_accept_le": ("pick = mulhi64(out[1], T) < prob[c]", "pick = mulhi64(out[1], T) <= prob[c]"),
    "rjs_accept_le": ("if (mulhi64(out[1], wmax) < w[c]) return", "if (mulhi64(out[1], wmax) <= w[c]) return"),
    "rjs_trial_key": ("uint64_t ctr[4] = {task, k, 0, 3};", "uint64_t ctr[4] = {task, 0, k, 3};"),
    "walk_ids_key": ("starts[qids[j]], qids[j], length", "starts[qids[j]], j, length"),
    "walk_ids_start": ("FWO_SAMPLER_ITS, starts[qids[j]], qids[j]", "FWO_SAMPLER_ITS, starts[j], qids[j]"),
    "padding": ("for (uint32_t s = t + 1; s <= length; ++s)", "for (uint32_t s = t + 1; s < length; ++s)"),
}


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, mutant_dir, monkeypatch):
    old, new = MUTANTS[name]
    text = SRC.read_text()
    assert text.count(old) >= 1, name
    src = mutant_dir / f"{name}.c"
    src.write_text(text.replace(old, new))
    (mutant_dir / "fw_oracle.h").write_text((SRC.parent / "fw_oracle.h").read_text())
    so = mutant_dir / f"lib{name}.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", str(src), "-o", str(so)],
                   check=True)
    monkeypatch.setattr(oracle, "_lib", oracle.bind(ctypes.CDLL(str(so))))
    failed = []
    ordered = [p for p in P.ALL_PINS if p not in P.SLOW_PINS] + [P.pin_invariants_rmat12] + \
        P.SLOW_PINS
    for pin in ordered:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
            break
    assert failed, f"mutant {name} passed every pin"
