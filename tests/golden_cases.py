"""Loader for the hand-worked fixtures in tests/golden/.

Trees are written as s-expressions and parsed here into the flattened prefix
byte format (one opcode per node, Section 3.1); numbers are exact decimal or
hex-float strings, and a fixture input that would round on the way to
binary32 is rejected, so every stored value is the hand-worked one.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

FLOAT_OPS = {"+": 0x80, "-": 0x81, "*": 0x82, "%": 0x83}
BOOL_OPS = {"and": 0x80, "or": 0x81, "nand": 0x82, "nor": 0x83}


def parse_tree(text: str, boolean: bool = False) -> np.ndarray:
    ops = BOOL_OPS if boolean else FLOAT_OPS
    toks = text.replace("(", " ( ").replace(")", " ) ").split()
    out: list[int] = []
    pos = 0

    def node():
        nonlocal pos
        tok = toks[pos]
        pos += 1
        if tok == "(":
            name = toks[pos]
            pos += 1
            out.append(ops[name])
            node()
            node()
            assert toks[pos] == ")", text
            pos += 1
        else:
            assert tok[0] == "x", tok
            out.append(int(tok[1:]))

    node()
    assert pos == len(toks), f"trailing tokens in {text!r}"
    return np.array(out, dtype=np.uint8)


def num(s: str) -> float:
    s = s.strip()
    if "0x" in s.lower():
        return float.fromhex(s)
    return float(s)


def f32(values) -> np.ndarray:
    v = [num(s) for s in values]
    a = np.array(v, dtype=np.float32)
    for want, got in zip(v, a):
        assert (math.isnan(want) and np.isnan(got)) or float(got) == want, f"{want!r} is not a binary32 value"
    return a


def words(values) -> np.ndarray:
    return np.array([int(s, 16) for s in values], dtype=np.uint64)


def valid_mask(W: int, T: int) -> np.ndarray:
    m = np.full(W, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    if T % 64:
        m[-1] = np.uint64((1 << (T % 64)) - 1)
    return m


def same_fitness(a: float, b: float) -> bool:
    return (math.isnan(a) and math.isnan(b)) or a == b


def load(name: str = "hand_worked.json") -> dict:
    with open(os.path.join(HERE, name)) as fh:
        return json.load(fh)
