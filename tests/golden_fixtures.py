"""Reader for the hand-derived fixtures in tests/golden/ (text: a graph, then
queries with their expected distances and hop counts).  Parsing only: the
expected values are the ones written in the files, with their derivations."""
import os
import struct

import numpy as np

import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
INF_U32 = 0xFFFFFFFF
INF_F32_BITS = 0x7F7FFFFF  # "inf" in a binary32 file: unreachable, held as the largest finite value


def names():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))


def _f32_bits(tok):
    b = struct.unpack("<I", struct.pack("<f", float.fromhex(tok)))[0]
    assert struct.unpack("<f", struct.pack("<I", b))[0] == float.fromhex(tok), "value not binary32: " + tok
    return b


def load(name):
    """Returns (graph, [(source, dist_bits uint32[n], hops uint32[n]), ...])."""
    n, wtype, arcs, queries = None, None, [], []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            key, rest = line[0], line[1:]
            if key == "n":
                n = int(rest[0])
            elif key == "weights":
                wtype = {"u32": gg.W_U32, "f32": gg.W_F32}[rest[0]]
            elif key == "arc":
                w = float.fromhex(rest[2]) if wtype == gg.W_F32 else int(rest[2])
                arcs.append((int(rest[0]), int(rest[1]), w))
            elif key == "query":
                queries.append([int(rest[0]), None, None])
            elif key in ("dist", "hops"):
                assert len(rest) == n, (name, key)
                if key == "dist" and wtype == gg.W_F32:
                    vals = [INF_F32_BITS if t == "inf" else _f32_bits(t) for t in rest]
                else:
                    vals = [INF_U32 if t == "inf" else int(t) for t in rest]
                queries[-1][1 if key == "dist" else 2] = np.array(vals, dtype=np.uint32)
            else:
                raise ValueError("%s: unknown line %r" % (name, key))
    g = gg.from_arcs(n, arcs, wtype=wtype, name=name[:-4])
    assert all(q[1] is not None and q[2] is not None for q in queries), name
    return g, [tuple(q) for q in queries]
