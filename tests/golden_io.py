"""Readers for the hand-worked fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for raw in fh:
            s = raw.strip()
            if s and not s.startswith("#"):
                yield s.split()


def fig3():
    d = {}
    for parts in lines("fig3_reduction.txt"):
        d[parts[0]] = [int(x) for x in parts[1:]]
    return d


def dff_values():
    return [(p[0], int(p[1]), int(p[2]), int(p[3]), int(p[4]), p[5] if len(p) > 5 else "") for p in lines("dff_values.txt")]


def hand_bounds():
    return [(p[0], int(p[1]), int(p[2]), int(p[3]), int(p[4]), [int(x) for x in p[5:]]) for p in lines("hand_bounds.txt")]


def param_counts():
    return [tuple(int(x) for x in p) for p in lines("param_counts.txt")]


def vb2_clamp():
    return [tuple(int(x) for x in p) for p in lines("vb2_clamp.txt")]
