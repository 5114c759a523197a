"""The partition enumerator against brute force over all set partitions of
small random scripts, filtered by a legality predicate written here from the
rules of Section 3.2 (independently of the library's implementation)."""
import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import randscript as R

RED = {"dot", "gemv", "gemtv"}
MAT = {"gemv", "gemtv", "ger"}


def structure(s):
    n = kf.kf_script_num_calls(s)
    calls = [kf.kf_script_call(s, i) for i in range(n)]
    producer = {c["out"]: i for i, c in enumerate(calls)}
    kinds = {}
    for i, c in enumerate(calls):
        for v in c["in"]:
            if v >= 0:
                kinds[v] = kf.kf_value_info(s, v)
        kinds[c["out"]] = kf.kf_value_info(s, c["out"])
    return calls, producer, kinds


def space(calls, kinds, i):
    c = calls[i]
    k = kinds[c["in"][0]]
    return ("m", k[1], k[2]) if c["op"] in MAT else ("v", k[1])


def deps(calls, producer):
    """edges producer -> consumer over every operand (scalars included)."""
    e = set()
    for j, c in enumerate(calls):
        for v in [c["alpha"], c["beta"]] + c["in"]:
            if v in producer:
                e.add((producer[v], j))
    return e


def legal_block(block, calls, producer, kinds):
    if len({space(calls, kinds, i) for i in block}) != 1:
        return False
    inb = set(block)
    for i in block:
        if calls[i]["op"] not in RED:
            continue
        out = calls[i]["out"]
        for j in block:
            c = calls[j]
            uses = [out == c["alpha"], out == c["beta"], out == c["in"][0], out == c["in"][1], out == c["in"][2]]
            if not any(uses):
                continue
            only_y0 = uses[4] and not any(uses[:4])
            if only_y0 and c["op"] == calls[i]["op"] and c["op"] in ("gemv", "gemtv"):
                continue
            # a row dot may feed a gemtv's row-indexed x when whole rows stay in
            # one workgroup (row-resident schedule, at most 32768 columns)
            only_x = uses[3] and not (uses[0] or uses[1] or uses[2] or uses[4])
            if calls[i]["op"] == "gemv" and c["op"] == "gemtv" and only_x and kinds[c["in"][0]][2] <= 32768:
                continue
            return False
    if len(block) > 1:
        data = []
        for i in block:
            c = calls[i]
            vs = {v for v in c["in"] + [c["out"]] if v >= 0 and kinds[v][0] in (0, 1)}
            data.append(vs)
        seen, stack = {0}, [0]
        while stack:
            a = stack.pop()
            for b in range(len(block)):
                if b not in seen and data[a] & data[b]:
                    seen.add(b)
                    stack.append(b)
        if len(seen) != len(block):
            return False
    return True


def acyclic(part, edges):
    k = max(part) + 1
    succ = {i: set() for i in range(k)}
    for a, b in edges:
        if part[a] != part[b]:
            succ[part[a]].add(part[b])
    state = {}

    def dfs(u):
        state[u] = 1
        for v in succ[u]:
            if state.get(v) == 1 or (v not in state and not dfs(v)):
                return False
        state[u] = 2
        return True

    return all(state.get(u) == 2 or dfs(u) for u in range(k))


def set_partitions(n):
    def rec(i, part, k):
        if i == n:
            yield list(part)
            return
        for b in range(k + 1):
            part.append(b)
            yield from rec(i + 1, part, max(k, b + 1))
            part.pop()
    yield from rec(0, [], 0)


def brute(s):
    calls, producer, kinds = structure(s)
    edges = deps(calls, producer)
    out = set()
    for part in set_partitions(len(calls)):
        blocks = {}
        for i, b in enumerate(part):
            blocks.setdefault(b, []).append(i)
        if all(legal_block(b, calls, producer, kinds) for b in blocks.values()) and acyclic(part, edges):
            out.add(tuple(part))
    return out


@pytest.mark.parametrize("seed", list(range(12)))
def test_enumerator_equals_bruteforce(seed):
    rs = R.random_script(1000 + seed, min_calls=5, max_calls=8, mat_log2=(6, 7), vec_log2=(6, 8))
    got = {tuple(p) for p in kf.kf_enumerate(rs.script, 0)}
    want = brute(rs.script)
    assert got == want, (rs.describe(), len(got), len(want))


def test_paper_sequences_bruteforce():
    from paper_1305_1183_amd import sequences as S
    for q in (S.gemver(64, 64, 1.5, 0.5), S.bicgk(64, 48), S.atax(32, 16), S.gesummv(32, 16, 1.5, 0.5),
              S.axpydot(1000, 1.5), S.waxpby(1000, 1.5, 0.5)):
        assert {tuple(p) for p in kf.kf_enumerate(q.script, 0)} == brute(q.script)
