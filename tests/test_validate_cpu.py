"""The plan validator (OBK_VALIDATE=1 inside obk_plan; obk_validate_layout_host
on host arrays) accepts the group-major layout of the oracle's plans and
names each planted mistake: a conflicting pair placed in one group, an entry
missing from its column, a value that differs between the row and column
copies, a row laid out in another group, columns out of order.  No device
is used."""
import numpy as np
import pytest

import oracle
import synth
import paper_2401_00672_amd as obk


def _layout(pl, group):
    """Group-major rows (ascending within each group), their CSR, and the
    per-group column segments, from a reordered CSR and a group per row."""
    n, G = pl.n, int(group.max()) + 1
    grow = np.array([i for g in range(G) for i in range(n) if group[i] == g], dtype=np.int32)
    gptr = np.zeros(G + 1, np.int64)
    np.add.at(gptr, group[group >= 0] + 1, 1)
    gptr = np.cumsum(gptr)
    rptr, rcol, rval = [0], [], []
    for i in grow:
        rcol += list(pl.ci[pl.rp[i]:pl.rp[i + 1]])
        rval += list(pl.v[pl.rp[i]:pl.rp[i + 1]])
        rptr.append(len(rcol))
    rptr = np.array(rptr, np.int64)
    tptr, tcol, sptr, srow, sval = [0], [], [0], [], []
    for g in range(G):
        ents = sorted((rcol[e], a, rval[e]) for a in range(gptr[g], gptr[g + 1]) for e in range(rptr[a], rptr[a + 1]))
        cols = sorted(set(c for c, _, _ in ents))
        for c in cols:
            tcol.append(c)
            for cc, a, v in ents:
                if cc == c:
                    srow.append(a)
                    sval.append(v)
            sptr.append(len(srow))
        tptr.append(len(tcol))
    return dict(n=n, gptr=gptr, grow=grow, group_of_row=np.asarray(group, np.int32), rptr=rptr,
                rcol=np.array(rcol, np.int32), rval=np.array(rval), tptr=np.array(tptr, np.int64),
                tcol=np.array(tcol, np.int32), sptr=np.array(sptr, np.int64), srow=np.array(srow, np.int32),
                sval=np.array(sval))


def _plan():
    s = synth.c2(grid=12)
    return oracle.plan_system(s, 0.1)


def test_validator_accepts_the_oracle_layouts():
    for s, delta in ((synth.c2(grid=12), 0.1), (synth.c1(n=300), 0.1), (synth.c1(n=200), 0.4)):
        pl = oracle.plan_system(s, delta)
        obk.validate_layout_host(**_layout(pl, pl.group), delta=delta)


def test_validator_names_a_conflict_inside_a_group():
    pl = _plan()
    # a conflicting pair: row i and a row j < i in its conflict list
    i = next(i for i in range(pl.n) if pl.cptr[i + 1] > pl.cptr[i])
    j = int(pl.cidx[pl.cptr[i]])
    g = pl.group.copy()
    g[i] = g[j]
    with pytest.raises(obk.ObkError) as e:
        obk.validate_layout_host(**_layout(pl, g), delta=0.1)
    assert e.value.code == -1 and "|cos|" in str(e.value)


@pytest.mark.parametrize("mistake,message", [
    ("drop_column_entry", "missing from its column"),
    ("column_value", "another value"),
    ("row_in_wrong_group", "belongs to"),
    ("columns_unsorted", "not ascending"),
])
def test_validator_names_planted_layout_mistakes(mistake, message):
    pl = _plan()
    L = _layout(pl, pl.group)
    if mistake == "drop_column_entry":
        # a segment with two rows loses its second entry
        seg = next(sg for sg in range(len(L["tcol"])) if L["sptr"][sg + 1] - L["sptr"][sg] >= 2)
        k = int(L["sptr"][seg]) + 1
        L["srow"] = np.delete(L["srow"], k)
        L["sval"] = np.delete(L["sval"], k)
        L["sptr"] = L["sptr"].copy()
        L["sptr"][seg + 1:] -= 1
    elif mistake == "column_value":
        L["sval"] = L["sval"].copy()
        L["sval"][3] = L["sval"][3] * (1 + 2 ** -40)
    elif mistake == "row_in_wrong_group":
        # the first row of group 1 names a row of group 0
        L["grow"] = L["grow"].copy()
        L["grow"][int(L["gptr"][1])] = L["grow"][0]
    elif mistake == "columns_unsorted":
        L["rcol"] = L["rcol"].copy()
        a = next(a for a in range(len(L["rptr"]) - 1) if L["rptr"][a + 1] - L["rptr"][a] >= 2)
        e = int(L["rptr"][a])
        L["rcol"][e], L["rcol"][e + 1] = L["rcol"][e + 1], L["rcol"][e]
    with pytest.raises(obk.ObkError) as ex:
        obk.validate_layout_host(**L, delta=0.1)
    assert ex.value.code == -1 and message in str(ex.value), str(ex.value)
