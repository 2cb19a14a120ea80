"""Independent recounts of an exported LD-Leiden state (numpy only).

Given a state dict {top, m, Ein, SKK, Kout, Kin, levels: [ {alive, lab, par, kout, kin, rows,
cols, w} ]} -- exported by either the oracle or the GPU library -- recompute from scratch:

  I1  W_{r+1}(x,y) = sum over pi_r(u)=x, pi_r(v)=y of W_r(u,v)   (paper Eq. 3) and liveness
  I2  P^r(u) = P^{r+1}(pi_r(u))                                  (labels nest)
  I3  a live level-(r+1) node x has its root node x at level r with pi_r(x) = x
  I4  every refined community is weakly connected in G^r
  I5  community totals, m, Ein and sum Kout*Kin from the level-0 matrix and P^0
  I6  degrees are row / column sums at every level
"""
from __future__ import annotations

import numpy as np


def _keys(rows, cols):
    return (rows.astype(np.uint64) << np.uint64(32)) | cols.astype(np.uint64)


def check_state(st: dict, directed: bool, check_connectivity: bool = True) -> list[str]:
    errs: list[str] = []
    top = st["top"]
    lv = st["levels"]
    n = len(lv[0]["lab"])
    for r in range(top + 1):
        L = lv[r]
        rows, cols, w = L["rows"], L["cols"], L["w"]
        if len(w) and w.min() <= 0:
            errs.append(f"level {r}: non-positive weight")
        alive = L["alive"].astype(bool)
        if len(rows) and (not alive[rows].all() or not alive[cols].all()):
            errs.append(f"level {r}: entry at a dead node")
        ko = np.zeros(n, dtype=np.int64)
        np.add.at(ko, rows, w)
        ki = np.zeros(n, dtype=np.int64)
        np.add.at(ki, cols, w)
        if not np.array_equal(ko, L["kout"]) or not np.array_equal(ki, L["kin"]):
            errs.append(f"level {r}: degree sums differ (I6)")
        k = _keys(rows, cols)
        if len(np.unique(k)) != len(k):
            errs.append(f"level {r}: duplicate entries")
        if not directed:
            kt = _keys(cols, rows)
            o1, o2 = np.argsort(k), np.argsort(kt)
            if not (np.array_equal(k[o1], kt[o2]) and np.array_equal(w[o1], w[o2])):
                errs.append(f"level {r}: undirected matrix not symmetric")
        if r < top:
            H = lv[r + 1]
            par = L["par"]
            live_par = np.zeros(n, dtype=bool)
            live_par[par[alive]] = True
            if not np.array_equal(live_par, H["alive"].astype(bool)):
                errs.append(f"level {r + 1}: liveness differs from parents (I1)")
            ak = _keys(par[rows], par[cols])
            uk, inv = np.unique(ak, return_inverse=True)
            s = np.zeros(len(uk), dtype=np.int64)
            np.add.at(s, inv, w)
            nz = s != 0
            uk, s = uk[nz], s[nz]
            hk = _keys(H["rows"], H["cols"])
            o = np.argsort(hk)
            if not (np.array_equal(uk, hk[o]) and np.array_equal(s, H["w"][o])):
                errs.append(f"level {r + 1}: aggregate differs from grouped sum of level {r} (I1)")
            au = np.nonzero(alive)[0]
            if not np.array_equal(L["lab"][au], H["lab"][par[au]]):
                errs.append(f"level {r}: labels do not nest (I2)")
            hx = np.nonzero(H["alive"])[0]
            if not (alive[hx].all() and np.array_equal(par[hx], hx)):
                errs.append(f"level {r}: refined community without its root (I3)")
            if check_connectivity:
                bad = _disconnected_refined(n, alive, par, rows, cols)
                if bad:
                    errs.append(f"level {r}: {bad} refined communities not connected (I4)")
    # I5 from the level-0 matrix and P^0
    L0 = lv[0]
    lab = L0["lab"]
    rows, cols, w = L0["rows"], L0["cols"], L0["w"]
    m = int(w.sum())
    Ko = np.zeros(n, dtype=np.int64)
    Ki = np.zeros(n, dtype=np.int64)
    np.add.at(Ko, lab[rows], w)
    np.add.at(Ki, lab[cols], w)
    ein = int(w[lab[rows] == lab[cols]].sum())
    skk = sum(int(a) * int(b) for a, b in zip(Ko[Ko != 0], Ki[Ko != 0]))
    if m != st["m"]:
        errs.append("m differs from recount (I5)")
    if ein != st["Ein"]:
        errs.append("Ein differs from recount (I5)")
    if not (np.array_equal(Ko, st["Kout"]) and np.array_equal(Ki, st["Kin"])):
        errs.append("community totals differ from recount (I5)")
    if skk != st["SKK"]:
        errs.append("sum Kout*Kin differs from recount (I5)")
    return errs


def _disconnected_refined(n, alive, par, rows, cols) -> int:
    """Count refined communities (alive nodes sharing pi) that are not weakly connected by the
    level's entries between members."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    same = par[rows] == par[cols]
    g = coo_matrix((np.ones(int(same.sum()), dtype=np.int8), (rows[same], cols[same])), shape=(n, n))
    _, comp = connected_components(g, directed=True, connection="weak")
    au = np.nonzero(alive)[0]
    pairs = np.unique((par[au].astype(np.uint64) << np.uint64(32)) | comp[au].astype(np.uint64))
    groups = pairs >> np.uint64(32)
    return int(len(groups) - len(np.unique(groups)))


def oracle_state(o) -> dict:
    sc = o.scalars()
    ko, ki = o.totals()
    return {"top": sc["top"], "m": sc["m"], "Ein": sc["Ein"], "SKK": sc["SKK"], "Kout": ko, "Kin": ki,
            "levels": [o.level(r) for r in range(sc["top"] + 1)]}


def diff_states(a: dict, b: dict) -> list[str]:
    """Bit-exact comparison of two exported states (par compared on alive nodes below top)."""
    d = []
    for k in ("top", "m", "Ein", "SKK"):
        if a[k] != b[k]:
            d.append(f"{k}: {a[k]} != {b[k]}")
    for k in ("Kout", "Kin"):
        if not np.array_equal(a[k], b[k]):
            d.append(f"{k} differs at {int(np.count_nonzero(a[k] != b[k]))} communities")
    if a["top"] != b["top"]:
        return d
    for r in range(a["top"] + 1):
        A, B = a["levels"][r], b["levels"][r]
        al = A["alive"].astype(bool)
        if not np.array_equal(al, B["alive"].astype(bool)):
            d.append(f"level {r}: alive differs")
            continue
        for k in ("lab", "kout", "kin"):
            if not np.array_equal(A[k][al], B[k][al]):
                d.append(f"level {r}: {k} differs at {int(np.count_nonzero(A[k][al] != B[k][al]))} nodes")
        if r < a["top"] and not np.array_equal(A["par"][al], B["par"][al]):
            d.append(f"level {r}: par differs at {int(np.count_nonzero(A['par'][al] != B['par'][al]))} nodes")
        ka, kb = _keys(A["rows"], A["cols"]), _keys(B["rows"], B["cols"])
        oa, ob = np.argsort(ka), np.argsort(kb)
        if not (np.array_equal(ka[oa], kb[ob]) and np.array_equal(A["w"][oa], B["w"][ob])):
            d.append(f"level {r}: matrix entries differ")
    return d


def state_digest(st: dict) -> dict:
    """SHA-256 digests of an exported state, field by field, in the comparison of diff_states
    (node arrays on alive nodes, parents below the top level, matrix entries in key order), plus
    a few plain values for reading a mismatch."""
    import hashlib

    def h(*arrs):
        d = hashlib.sha256()
        for a in arrs:
            d.update(np.ascontiguousarray(a).tobytes())
        return d.hexdigest()[:32]

    out = {"top": int(st["top"]), "m": int(st["m"]), "Ein": int(st["Ein"]), "SKK": str(int(st["SKK"])),
           "Kout": h(st["Kout"].astype("<i8")), "Kin": h(st["Kin"].astype("<i8")), "levels": []}
    for r, L in enumerate(st["levels"]):
        al = L["alive"].astype(bool)
        k = _keys(L["rows"], L["cols"])
        w = L["w"].astype("<i8")
        if len(k) > 1 and not bool(np.all(k[1:] > k[:-1])):
            o = np.argsort(k, kind="stable")
            k, w = k[o], w[o]
        lv = {"alive": h(L["alive"].astype(np.uint8)), "n_alive": int(al.sum()), "lab": h(L["lab"][al].astype("<u4")),
              "kout": h(L["kout"][al].astype("<i8")), "kin": h(L["kin"][al].astype("<i8")), "nnz": int(len(k)),
              "entries": h(k.astype("<u8"), w)}
        if r < st["top"]:
            lv["par"] = h(L["par"][al].astype("<u4"))
        out["levels"].append(lv)
    lab0 = st["levels"][0]["lab"]
    out["communities"] = int(len(np.unique(lab0)))
    out["labels_head"] = [int(x) for x in lab0[:8]]
    return out


def digest_diff(a: dict, b: dict) -> list[str]:
    """Fields in which two state digests differ."""
    d = []
    for k in ("top", "m", "Ein", "SKK", "Kout", "Kin", "communities", "labels_head"):
        if a.get(k) != b.get(k):
            d.append(f"{k}: {a.get(k)} != {b.get(k)}")
    for r, (x, y) in enumerate(zip(a["levels"], b["levels"])):
        for k in sorted(set(x) | set(y)):
            if x.get(k) != y.get(k):
                d.append(f"level {r} {k}: {x.get(k)} != {y.get(k)}")
    return d
