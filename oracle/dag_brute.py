"""Literal brute force of the STF dependency definition, for tiny programs only.

Test infrastructure: used to check the oracle's C edge enumeration.

STF (Specx, Sec. 2.1 and Sec. 4.1): tasks are inserted in program order with SpRead
(read-only) or SpWrite (read-or-write) accesses; the order of insertion fixes the
read-after-write and write-after-read dependencies.  For tasks a < b, edge (a,b) exists
iff some datum d is used by both with at least one write and
  RAW: a writes d, b only reads d, and no task strictly between them writes d;
  WAR: a only reads d, b writes d, and no task strictly between them writes d;
  WAW: both write d, and no task strictly between them reads or writes d.
This walks every pair of tasks and every datum, with no per-datum bookkeeping.
"""

R, RW = 1, 2


def modes_by_task(ntasks, accesses):
    """accesses: iterable of (task, mode, datum) -> list of {datum: mode} per task."""
    per = [dict() for _ in range(ntasks)]
    for t, m, d in accesses:
        per[t][d] = RW if (m == RW or per[t].get(d) == RW) else R
    return per


def edges(ntasks, accesses):
    """Returns (sorted list of (a, b), {'RAW': n, 'WAR': n, 'WAW': n})."""
    per = modes_by_task(ntasks, accesses)
    data = sorted({d for p in per for d in p})
    out = set()
    kinds = {"RAW": set(), "WAR": set(), "WAW": set()}
    for a in range(ntasks):
        for b in range(a + 1, ntasks):
            for d in data:
                ma, mb = per[a].get(d), per[b].get(d)
                if ma is None or mb is None or (ma == R and mb == R):
                    continue
                between = [per[t].get(d) for t in range(a + 1, b)]
                any_write = any(m == RW for m in between)
                any_use = any(m is not None for m in between)
                if ma == RW and mb == R and not any_write:
                    kind = "RAW"
                elif ma == R and mb == RW and not any_write:
                    kind = "WAR"
                elif ma == RW and mb == RW and not any_use:
                    kind = "WAW"
                else:
                    continue
                out.add((a, b))
                kinds[kind].add((a, b))
    return sorted(out), {k: len(v) for k, v in kinds.items()}


def conflict_closure(ntasks, accesses):
    """Transitive closure of the FULL conflict relation: (a,b), a<b, share a datum with
    at least one write.  Returned as a set of pairs."""
    per = modes_by_task(ntasks, accesses)
    conf = [set() for _ in range(ntasks)]
    for a in range(ntasks):
        for b in range(a + 1, ntasks):
            for d, ma in per[a].items():
                mb = per[b].get(d)
                if mb is not None and (ma == RW or mb == RW):
                    conf[a].add(b)
                    break
    return closure(ntasks, [(a, b) for a in range(ntasks) for b in conf[a]])


def closure(ntasks, edge_list):
    succ = [[] for _ in range(ntasks)]
    for a, b in edge_list:
        succ[a].append(b)
    reach = [set() for _ in range(ntasks)]
    for a in range(ntasks - 1, -1, -1):  # edges point forward: process in reverse
        for b in succ[a]:
            reach[a].add(b)
            reach[a] |= reach[b]
    return {(a, b) for a in range(ntasks) for b in reach[a]}


CW = 3
GROUP_MAX = 63


def commutative_groups(ntasks, accesses):
    """Per task, {datum: group id} for its commutative writes: on each datum, a run of
    consecutive commutative writes (no other use of the datum between them, counting in
    insertion order) forms a group, cut every GROUP_MAX members."""
    per = [dict() for _ in range(ntasks)]
    for t, m, d in accesses:
        old = per[t].get(d)
        per[t][d] = m if old is None or old == m else RW
    groups = [dict() for _ in range(ntasks)]
    data = sorted({d for p in per for d in p})
    gid = 0
    for d in data:
        users = [t for t in range(ntasks) if d in per[t]]
        run = 0
        prev_cw = False
        for t in users:
            if per[t][d] == CW:
                if not prev_cw or run == GROUP_MAX:
                    gid += 1
                    run = 0
                groups[t][d] = gid
                run += 1
                prev_cw = True
            else:
                prev_cw = False
    return per, groups


def commutative_conflict_closure(ntasks, accesses):
    """Transitive closure of the order a parallel run must keep (Specx Sec. 4.1): tasks a < b
    sharing a datum that at least one of them writes, unless both are commutative writes
    of the same group (those may run in either order).  A set of pairs."""
    per, groups = commutative_groups(ntasks, accesses)
    pairs = []
    for a in range(ntasks):
        for b in range(a + 1, ntasks):
            for d, ma in per[a].items():
                mb = per[b].get(d)
                if mb is None or (ma == R and mb == R):
                    continue
                if ma == CW and mb == CW and groups[a][d] == groups[b][d]:
                    continue
                pairs.append((a, b))
                break
    return closure(ntasks, pairs)
