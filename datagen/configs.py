"""Seeded synthetic workloads shaped like the paper's (Section 4, Tables 1-2).

The paper measures on Retailer, Favorita, Yelp and TPC-DS, none of which is
available here; these relations stand in for them: a large fact table sorted
by its foreign keys (Appendix B: relations are given sorted by their join
attributes; Section 3.5 orders join attributes by increasing domain size),
small dimension tables with dense unique keys, continuous and categorical
attributes, 20-bucket discretisation of continuous attributes for decision
trees (Appendix B), and batches of the paper's application families
(Section 2: covariance matrix, regression-tree node, mutual information).

Five workloads (all sizes are parameters; defaults are the full sizes):

1. tiny star, 100k facts: covariance of 9 attributes plus one grouped sum;
2. snowflake, 10M facts, Zipf(1.1) keys: ridge-regression batch with
   categorical group-bys and pairwise categorical counts;
3. regression-tree level, 50M facts: COUNT, SUM(y), SUM(y^2) grouped by
   (node, attribute, bucket) for 32 random nodes;
4. covariance batch, 100M facts, Zipf(1.2) keys, values N(100, 1);
5. mutual-information counts, 50M facts, 15 categorical attributes.

Every column is a pure function of (seed, relation, column, row).  Fact
foreign-key tuples are drawn per row, sorted lexicographically (smallest
dimension first), and the remaining fact attributes are then drawn by sorted
row index; since rows are i.i.d. this equals drawing then sorting.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .rng import native
from .schema import Agg, Column, Database, GroupBy, Pred, Query, Relation


# ---------------------------------------------------------------------------
# relation recipes
# ---------------------------------------------------------------------------

@dataclass
class AttrSpec:
    name: str
    kind: str                      # "cont" | "cat"
    dist: Tuple = ("normal", 0.0, 1.0)   # cont: ("normal", m, sd) | ("uniform", lo, hi)
    domain: int = 0                # cat: codes uniform in [0, domain)


@dataclass
class RelSpec:
    name: str
    n_rows: int
    attrs: List[AttrSpec]
    key: Optional[str] = None                 # primary key attribute (dims)
    children: List[Tuple["RelSpec", str]] = field(default_factory=list)   # (child, key dist)
    zipf_s: Dict[str, float] = field(default_factory=dict)                # per FK: Zipf exponent


def zipf_cdf(n: int, s: float) -> np.ndarray:
    """Bounded Zipf over ranks 1..n, P(r) proportional to r^-s; rank r -> key r-1."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w) / w.sum()
    cdf[-1] = 1.0
    return cdf


def _draw_attr(seed: int, rel: str, a: AttrSpec, n: int) -> Column:
    g = native()
    key = g.key(seed, "%s.%s" % (rel, a.name))
    if a.kind == "cont":
        if a.dist[0] == "normal":
            data = g.normal_f32(key, n, a.dist[1], a.dist[2])
        elif a.dist[0] == "uniform":
            data = g.uniform_f32(key, n, a.dist[1], a.dist[2])
        else:
            raise ValueError(a.dist)
        return Column(a.name, "cont", data)
    if a.kind == "cat":
        return Column(a.name, "cat", g.uniform_i32(key, n, 0, a.domain), a.domain)
    raise ValueError(a.kind)


def _draw_fk(seed: int, rel: str, fk: str, n: int, domain: int, s: float) -> np.ndarray:
    g = native()
    key = g.key(seed, "%s.%s" % (rel, fk))
    if s > 0.0:
        return g.from_cdf_i32(key, n, zipf_cdf(domain, s))
    return g.uniform_i32(key, n, 0, domain)


def build_relation(seed: int, spec: RelSpec, sort_fks: bool) -> Relation:
    """Draw one relation: its primary key (dense 0..n-1), foreign keys into its
    children, and its own attributes.  With ``sort_fks`` the foreign-key tuples
    are sorted lexicographically, smallest child domain first."""
    n = spec.n_rows
    cols: List[Column] = []
    if spec.key is not None:
        cols.append(Column(spec.key, "key", np.arange(n, dtype=np.int32), n))
    fks = []
    for child, fk in spec.children:
        s = spec.zipf_s.get(fk, 0.0)
        fks.append((fk, child.n_rows, _draw_fk(seed, spec.name, fk, n, child.n_rows, s)))
    if fks and sort_fks:
        order = sorted(range(len(fks)), key=lambda i: fks[i][1])
        radix = [fks[i][1] for i in order]
        if math.prod(radix) < 2 ** 63:
            g = native()
            comp = g.compose([fks[i][2] for i in order], radix)
            comp = g.sort_u64(comp)
            sorted_cols = g.decompose(comp, radix)
            del comp
            for j, i in enumerate(order):
                fks[i] = (fks[i][0], fks[i][1], sorted_cols[j])
        else:
            lead = order[0]
            perm = np.argsort(fks[lead][2], kind="stable")
            fks = [(a, d, v[perm]) for a, d, v in fks]
    for fk, dom, vals in fks:
        cols.append(Column(fk, "key", vals, dom))
    for a in spec.attrs:
        cols.append(_draw_attr(seed, spec.name, a, n))
    return Relation(spec.name, cols)


def build_database(seed: int, root: RelSpec) -> Database:
    rels: List[Relation] = []
    edges: List[Tuple[int, int]] = []

    def visit(spec: RelSpec, is_root: bool) -> int:
        idx = len(rels)
        rels.append(build_relation(seed, spec, sort_fks=is_root))
        for child, _fk in spec.children:
            c = visit(child, False)
            edges.append((idx, c))
        return idx

    visit(root, True)
    return Database(rels, edges)


def _domain_uniform(seed: int, name: str, lo: int, hi_incl: int) -> int:
    g = native()
    return int(g.uniform_i32(g.key(seed, "domain." + name), 1, lo, hi_incl + 1)[0])


def _domain_loguniform(seed: int, name: str, lo: int, hi: int) -> int:
    g = native()
    u = float(g.unit(g.key(seed, "domain." + name), 1)[0])
    return int(round(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))


def cont_attrs(db: Database) -> List[str]:
    """Continuous attributes in relation order (fact first)."""
    return [c.attr for r in db.relations for c in r.columns if c.kind == "cont"]


def cat_attrs(db: Database) -> List[str]:
    return [c.attr for r in db.relations for c in r.columns if c.kind == "cat"]


def covariance_queries(conts: Sequence[str]) -> List[Query]:
    """COUNT, SUM(x_i) and SUM(x_i * x_j) for i <= j, one query each
    (Section 2, covariance matrix; (n+1)(n+2)/2 aggregates for n attributes)."""
    qs = [Query()]
    qs += [Query(aggs=[Agg.monomial(a)]) for a in conts]
    for i in range(len(conts)):
        for j in range(i, len(conts)):
            qs.append(Query(aggs=[Agg.monomial(conts[i], conts[j])]))
    return qs


def polynomial_queries(conts: Sequence[str]) -> List[Query]:
    """Degree-2 polynomial regression (Section 2): the covariance matrix of the
    vector u = [1, x_i, x_i * x_j (i <= j)], one query per entry u_a * u_b with
    a <= b -- products of up to four attributes; (C^2 + C) / 2 aggregates for
    C = (n+1)(n+2)/2."""
    u: List[Tuple[str, ...]] = [()]
    u += [(a,) for a in conts]
    u += [(conts[i], conts[j]) for i in range(len(conts)) for j in range(i, len(conts))]
    qs = []
    for a in range(len(u)):
        for b in range(a, len(u)):
            f = u[a] + u[b]
            qs.append(Query() if not f else Query(aggs=[Agg.monomial(*f)]))
    return qs


# ---------------------------------------------------------------------------
# workload 1: tiny star
# ---------------------------------------------------------------------------

def config1(n_fact: int = 100_000, d1: int = 1000, d2: int = 500, seed: int = 1) -> Database:
    D1 = RelSpec("D1", d1, [AttrSpec("y%d" % i, "cont", ("uniform", 0.0, 1.0)) for i in (1, 2, 3)], key="a")
    D2 = RelSpec("D2", d2, [AttrSpec("z1", "cont"), AttrSpec("z2", "cont"),
                            AttrSpec("c", "cat", domain=10)], key="b")
    F = RelSpec("F", n_fact, [AttrSpec("x%d" % i, "cont") for i in (1, 2, 3, 4)],
                children=[(D1, "a"), (D2, "b")])
    return build_database(seed, F)


def batch1(db: Database) -> List[Query]:
    qs = covariance_queries(cont_attrs(db))
    qs.append(Query(groupby=[GroupBy("c")], aggs=[Agg.monomial("x1")]))
    return qs


# ---------------------------------------------------------------------------
# workload 2: snowflake, plain vs batched
# ---------------------------------------------------------------------------

def config2(n_fact: int = 10_000_000, dims: Sequence[int] = (10_000, 2_000, 50_000, 1_000),
            n_sub: int = 200, seed: int = 2) -> Database:
    def cat(name):
        return AttrSpec(name, "cat", domain=_domain_uniform(seed, name, 5, 200))

    S = RelSpec("S", n_sub, [AttrSpec("s1", "cont"), AttrSpec("s2", "cont"), cat("c3")], key="ks")
    D1 = RelSpec("D1", dims[0], [AttrSpec("d1_%d" % i, "cont") for i in range(1, 6)] + [cat("c1")], key="k1")
    D2 = RelSpec("D2", dims[1], [AttrSpec("d2_%d" % i, "cont") for i in range(1, 5)] + [cat("c2")], key="k2")
    D3 = RelSpec("D3", dims[2], [AttrSpec("d3_%d" % i, "cont") for i in range(1, 6)], key="k3",
                 children=[(S, "ks")])
    D4 = RelSpec("D4", dims[3], [AttrSpec("d4_%d" % i, "cont") for i in range(1, 5)] + [cat("c4")], key="k4")
    F = RelSpec("F", n_fact, [AttrSpec("f%d" % i, "cont") for i in range(1, 11)] + [cat("c0")],
                children=[(D1, "k1"), (D2, "k2"), (D3, "k3"), (D4, "k4")],
                zipf_s={"k1": 1.1, "k2": 1.1, "k3": 1.1, "k4": 1.1})
    return build_database(seed, F)


def batch2(db: Database) -> List[Query]:
    conts = cont_attrs(db)
    cats = sorted(cat_attrs(db))
    qs = covariance_queries(conts)
    for c in cats:
        qs += [Query(groupby=[GroupBy(c)], aggs=[Agg.monomial(x)]) for x in conts]
        qs.append(Query(groupby=[GroupBy(c)]))
    for i in range(len(cats)):
        for j in range(i + 1, len(cats)):
            qs.append(Query(groupby=[GroupBy(cats[i]), GroupBy(cats[j])]))
    return qs


# ---------------------------------------------------------------------------
# workload 3: regression-tree level
# ---------------------------------------------------------------------------

def config3(n_fact: int = 50_000_000, dims: Sequence[int] = (100_000, 5_000, 1_000), seed: int = 3) -> Database:
    def cat(name):
        return AttrSpec(name, "cat", domain=_domain_uniform(seed, name, 2, 100))

    def conts(prefix, n):
        return [AttrSpec("%s%d" % (prefix, i), "cont") for i in range(1, n + 1)]

    D1 = RelSpec("D1", dims[0], conts("u", 6) + [cat("a1"), cat("a2"), cat("a3")], key="k1")
    D2 = RelSpec("D2", dims[1], conts("v", 4) + [cat("b1"), cat("b2")], key="k2")
    D3 = RelSpec("D3", dims[2], conts("w", 2) + [cat("e1"), cat("e2")], key="k3")
    F = RelSpec("F", n_fact, [AttrSpec("y", "cont")] + conts("x", 8) + [cat("g1"), cat("g2"), cat("g3")],
                children=[(D1, "k1"), (D2, "k2"), (D3, "k3")])
    return build_database(seed, F)


def draw_thresholds(seed: int, attr: str, count: int = 20) -> np.ndarray:
    """``count`` distinct N(0,1) draws rounded to fp32, sorted ascending
    (duplicates are replaced by further draws of the same stream)."""
    g = native()
    key = g.key(seed, "thresholds." + attr)
    n = count
    while True:
        vals = g.normal_f64(key, n, 0.0, 1.0).astype(np.float32)
        uniq = []
        seen = set()
        for v in vals:
            if float(v) not in seen:
                seen.add(float(v))
                uniq.append(v)
            if len(uniq) == count:
                return np.sort(np.array(uniq, np.float32))
        n += count


@dataclass
class TreeLevel:
    features: List[str]                    # the 30 split attributes (20 continuous, 10 categorical)
    thresholds: Dict[str, np.ndarray]      # continuous attribute -> 20 thresholds
    nodes: List[List[Pred]]                # one conjunction per node


def tree_level(db: Database, n_nodes: int = 32, seed: int = 3) -> TreeLevel:
    conts = [a for a in cont_attrs(db) if a != "y"]
    cats = cat_attrs(db)
    feats = conts + cats
    th = {a: draw_thresholds(seed, a) for a in conts}
    g = native()
    nodes = []
    for n in range(n_nodes):
        u = g.unit(g.key(seed, "node%d" % n), 64)
        pos = 0

        def nxt():
            nonlocal pos
            pos += 1
            return float(u[pos - 1])

        k = 1 + min(int(nxt() * 5), 4)
        preds = []
        for _ in range(k):
            a = feats[min(int(nxt() * len(feats)), len(feats) - 1)]
            if a in th:
                op = "le" if nxt() < 0.5 else "gt"
                j = min(int(nxt() * 20), 19)
                preds.append(Pred(a, op, float(th[a][j])))
            else:
                dom = db.column(a).domain
                op = "eq" if nxt() < 0.5 else "ne"
                v = min(int(nxt() * dom), dom - 1)
                preds.append(Pred(a, op, float(v)))
        nodes.append(preds)
    return TreeLevel(feats, th, nodes)


def batch3(db: Database, level: Optional[TreeLevel] = None) -> List[Query]:
    """COUNT, SUM(y), SUM(y*y) GROUP BY bucket(attr), one query per
    (node, attribute) (Section 2, regression trees, equation (8))."""
    level = level or tree_level(db)
    qs = []
    for preds in level.nodes:
        for a in level.features:
            gb = GroupBy(a, level.thresholds.get(a))
            qs.append(Query(groupby=[gb], where=list(preds),
                            aggs=[Agg.monomial("y"), Agg.monomial("y", "y")]))
    return qs


def classification_tree_batch(db: Database, label: str, level: Optional[TreeLevel] = None) -> List[Query]:
    """Classification-tree level (Section 2, equations (9) and (10)): for every
    node (its conjunction of conditions as WHERE) and every split attribute X
    other than the label, COUNT GROUP BY (label, bucket(X)) and COUNT GROUP BY
    bucket(X).  The label's class frequencies per split condition follow from
    the pair, as the Gini index or entropy need."""
    level = level or tree_level(db)
    qs = []
    for preds in level.nodes:
        for a in level.features:
            if a == label:
                continue
            gb = GroupBy(a, level.thresholds.get(a))
            qs.append(Query(groupby=[GroupBy(label), gb], where=list(preds)))
            qs.append(Query(groupby=[gb], where=list(preds)))
    return qs


# ---------------------------------------------------------------------------
# data cube (Section 2, equation (6)) over workload 2's schema
# ---------------------------------------------------------------------------

def data_cube_batch(dims: Sequence[str], measures: Sequence[str]) -> List[Query]:
    """A k-dimensional data cube: one query per subset of the k dimensions
    (2^k group-bys, from the empty one to all k), each summing every measure
    (the paper's experiments use three dimensions and five measures)."""
    qs = []
    k = len(dims)
    for mask in range(1 << k):
        gb = [GroupBy(dims[i]) for i in range(k) if (mask >> i) & 1]
        qs.append(Query(groupby=gb, aggs=[Agg.monomial(m) for m in measures]))
    return qs


# ---------------------------------------------------------------------------
# workload 4: covariance batch (the headline measurement)
# ---------------------------------------------------------------------------

def config4(n_fact: int = 100_000_000, dims: Sequence[int] = (1_000_000, 100_000, 10_000, 1_000),
            seed: int = 4) -> Database:
    def conts(prefix, n):
        return [AttrSpec("%s%d" % (prefix, i), "cont", ("normal", 100.0, 1.0)) for i in range(1, n + 1)]

    Ds = [RelSpec("D%d" % (i + 1), dims[i], conts("d%d_" % (i + 1), 6), key="k%d" % (i + 1)) for i in range(4)]
    F = RelSpec("F", n_fact, conts("f", 16), children=[(D, D.key) for D in Ds],
                zipf_s={D.key: 1.2 for D in Ds})
    return build_database(seed, F)


def batch4(db: Database) -> List[Query]:
    return covariance_queries(cont_attrs(db))


# ---------------------------------------------------------------------------
# workload 5: pairwise counts for mutual information
# ---------------------------------------------------------------------------

def config5(n_fact: int = 50_000_000, dims: Sequence[int] = (100_000, 10_000, 1_000), seed: int = 5) -> Database:
    def cats(prefix, n):
        out = []
        for i in range(1, n + 1):
            name = "%s%d" % (prefix, i)
            out.append(AttrSpec(name, "cat", domain=_domain_loguniform(seed, name, 2, 1000)))
        return out

    Ds = [RelSpec("D%d" % (i + 1), dims[i], cats("m%d_" % (i + 1), 3), key="k%d" % (i + 1)) for i in range(3)]
    F = RelSpec("F", n_fact, cats("g", 6), children=[(D, D.key) for D in Ds])
    return build_database(seed, F)


def batch5(db: Database) -> List[Query]:
    """All marginal and pairwise COUNT GROUP BY queries over the categorical
    attributes (Section 2, mutual information, equation (7))."""
    cats = cat_attrs(db)
    qs = [Query(groupby=[GroupBy(c)]) for c in cats]
    for i in range(len(cats)):
        for j in range(i + 1, len(cats)):
            qs.append(Query(groupby=[GroupBy(cats[i]), GroupBy(cats[j])]))
    return qs


# ---------------------------------------------------------------------------
# registry
# ---------------------------------------------------------------------------

FULL = {
    1: dict(n_fact=100_000, d1=1000, d2=500),
    2: dict(n_fact=10_000_000, dims=(10_000, 2_000, 50_000, 1_000), n_sub=200),
    3: dict(n_fact=50_000_000, dims=(100_000, 5_000, 1_000)),
    4: dict(n_fact=100_000_000, dims=(1_000_000, 100_000, 10_000, 1_000)),
    5: dict(n_fact=50_000_000, dims=(100_000, 10_000, 1_000)),
}

# reduced sizes the oracle finishes in seconds; still many tiles plus a ragged tail
SMALL = {
    1: dict(n_fact=100_000, d1=1000, d2=500),
    2: dict(n_fact=200_003, dims=(1_000, 200, 5_000, 100), n_sub=20),
    3: dict(n_fact=100_003, dims=(2_000, 500, 100)),
    4: dict(n_fact=300_007, dims=(10_000, 1_000, 100, 10)),
    5: dict(n_fact=200_003, dims=(2_000, 500, 100)),
}

BUILDERS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


# ---------------------------------------------------------------------------
# many-to-many star (Yelp-like: reviews of businesses with several categories
# and attributes per business, Section 4)
# ---------------------------------------------------------------------------

def many_to_many_database(n_fact: int = 200_000, n_users: int = 5_000, n_business: int = 2_000,
                          mean_cat: int = 3, mean_attr: int = 2, seed: int = 11) -> Database:
    """Review(user, business) fact, Zipf(1.1) keys, sorted; User and Business
    dimensions with unique keys; Category and Attribute with, per business, a
    number of rows uniform in [0, 2 * mean] (businesses with none do not
    join), keyed by the repeated join attribute ``business``."""
    g = native()
    U = RelSpec("User", n_users, [AttrSpec("u1", "cont", ("normal", 3.0, 1.0)), AttrSpec("u2", "cont"),
                                  AttrSpec("ucat", "cat", domain=7)], key="user")
    B = RelSpec("Business", n_business, [AttrSpec("b1", "cont", ("uniform", 1.0, 5.0)),
                                         AttrSpec("bcat", "cat", domain=12)], key="business")
    F = RelSpec("Review", n_fact, [AttrSpec("stars", "cont", ("uniform", 1.0, 5.0)), AttrSpec("useful", "cont"),
                                   AttrSpec("rcat", "cat", domain=5)],
                children=[(U, "user"), (B, "business")], zipf_s={"user": 1.1, "business": 1.1})
    db = build_database(seed, F)
    many = [("Category", mean_cat, [AttrSpec("cw", "cont", ("normal", 2.0, 1.5)),
                                    AttrSpec("cv", "cont", ("uniform", -1.0, 1.0))]),
            ("Attribute", mean_attr, [AttrSpec("aw", "cont", ("normal", 0.0, 2.0))])]
    for name, mean, attrs in many:
        per_key = g.uniform_i32(g.key(seed, name + ".rows"), n_business, 0, 2 * mean + 1)
        keys = np.repeat(np.arange(n_business, dtype=np.int32), per_key.astype(np.int64))
        cols = [Column("business", "key_many", keys, n_business)]
        cols += [_draw_attr(seed, name, a, len(keys)) for a in attrs]
        db.relations.append(Relation(name, cols))
        db.edges.append((0, len(db.relations) - 1))
    return db


def many_to_many_batch(db: Database) -> List[Query]:
    """Covariance of every continuous attribute, grouped sums by categories of
    the other relations, and filtered sums of the many-to-many attributes."""
    conts = cont_attrs(db)
    qs = covariance_queries(conts)
    for c in ("bcat", "ucat", "rcat"):
        qs.append(Query(groupby=[GroupBy(c)], aggs=[Agg.monomial("cw"), Agg.monomial("aw"), Agg.monomial("stars", "cv"),
                                                    Agg.monomial("u1")]))
    qs.append(Query(groupby=[GroupBy("bcat"), GroupBy("rcat")]))
    qs.append(Query(where=[Pred("stars", "gt", 3.0)], aggs=[Agg.monomial("cw"), Agg.monomial("aw", "b1")]))
    qs.append(Query(groupby=[GroupBy("ucat")], where=[Pred("b1", "le", 2.5), Pred("rcat", "ne", 1)],
                    aggs=[Agg.monomial("cv"), Agg.monomial("useful")]))
    return qs


def many_to_many_local_queries() -> List[Query]:
    """Queries local to the many-to-many children of many_to_many_database: group-bys and
    predicates on their attributes, grouped products of two of them, three- and four-factor
    products, mixed with attributes of the other relations."""
    b3 = np.array([0.0, 1.5, 3.0], np.float32)
    return [
        Query(groupby=[GroupBy("cw", b3)], aggs=[Agg.monomial("stars"), Agg.monomial("cw"), Agg.monomial("u1", "cw")]),
        Query(groupby=[GroupBy("bcat"), GroupBy("cv", np.array([0.0], np.float32))],
              aggs=[Agg.monomial("cw", "cv"), Agg([(2.0, ("useful",)), (-1.0, ("cw", "b1"))])]),
        Query(where=[Pred("aw", "gt", 0.0)], aggs=[Agg.monomial("stars"), Agg.monomial("aw", "aw"), Agg.monomial("cw")]),
        Query(groupby=[GroupBy("ucat")], where=[Pred("cv", "le", 0.25), Pred("stars", "gt", 2.0)],
              aggs=[Agg.monomial("cv", "stars"), Agg.monomial("aw")]),
        Query(groupby=[GroupBy("rcat"), GroupBy("ucat")], where=[Pred("aw", "ne", 0.5)]),
        Query(aggs=[Agg.monomial("cw", "cv", "stars"), Agg.monomial("cw", "cw", "u1", "b1")]),
        Query(groupby=[GroupBy("aw", np.array([-1.0, 1.0], np.float32))], where=[Pred("b1", "gt", 2.0)],
              aggs=[Agg.monomial("aw", "cw")]),
    ]


def many_to_many_join_size(db: Database) -> int:
    """|J| of many_to_many_database: per review, the product of its business's category and
    attribute rows (users and businesses are unique keys covering every foreign key)."""
    b = db.rel("Review").col("business").data
    n = db.rel("Business").n_rows
    c = np.bincount(db.rel("Category").col("business").data, minlength=n).astype(np.int64)
    a = np.bincount(db.rel("Attribute").col("business").data, minlength=n).astype(np.int64)
    return int(np.sum(c[b] * a[b]))


def make_database(k: int, size: str = "small", **override) -> Database:
    params = dict((FULL if size == "full" else SMALL)[k])
    params.update(override)
    return BUILDERS[k](**params)


def make_batch(k: int, db: Database) -> List[Query]:
    if k == 1:
        return batch1(db)
    if k == 2:
        return batch2(db)
    if k == 3:
        return batch3(db, tree_level(db, seed=3))
    if k == 4:
        return batch4(db)
    if k == 5:
        return batch5(db)
    raise ValueError(k)


# ---------------------------------------------------------------------------
# random star/snowflake workloads (training and held-out data of the cost model)
# ---------------------------------------------------------------------------

def random_workload(j: int, max_rows: int = 20_000_000, min_rows: int = 1_000):
    """Random schema and batch number j (seed 6000 + j): 2-6 relations, each
    dimension attached to the fact or to an earlier dimension; sizes
    log-uniform in [min_rows, max_rows] with the fact largest; 1-10 continuous
    and 0-5 categorical attributes per relation; 10-500 aggregates mixing
    covariance entries, grouped sums, pairwise counts and filtered sums."""
    seed = 6000 + j
    g = native()
    u = g.unit(g.key(seed, "shape"), 4096)
    pos = [0]

    def nxt():
        pos[0] += 1
        return float(u[pos[0] - 1])

    def loguni(lo, hi):
        return int(round(math.exp(math.log(lo) + nxt() * (math.log(hi) - math.log(lo)))))

    m = 2 + min(int(nxt() * 5), 4)
    sizes = sorted([loguni(min_rows, max_rows) for _ in range(m)], reverse=True)
    specs = []
    for r in range(m):
        n_cont = 1 + min(int(nxt() * 10), 9)
        n_cat = min(int(nxt() * 6), 5)
        name = "F" if r == 0 else "R%d" % r
        attrs = [AttrSpec("%s_x%d" % (name, i), "cont") for i in range(n_cont)]
        attrs += [AttrSpec("%s_c%d" % (name, i), "cat", domain=2 + min(int(nxt() * 60), 59)) for i in range(n_cat)]
        specs.append(RelSpec(name, sizes[r], attrs, key=None if r == 0 else "k%d" % r))
    for r in range(1, m):
        parent = 0 if r == 1 or nxt() < 0.6 else 1 + min(int(nxt() * (r - 1)), r - 2)
        specs[parent].children.append((specs[r], "k%d" % r))
        if parent == 0 and nxt() < 0.5:
            specs[0].zipf_s["k%d" % r] = 1.1
    db = build_database(seed, specs[0])
    conts = cont_attrs(db)
    cats = cat_attrs(db)
    qs: List[Query] = []
    budget = 10 + min(int(nxt() * 491), 490)
    # covariance block over a random subset of continuous attributes
    k = max(1, min(len(conts), int(math.sqrt(2 * budget * nxt())) or 1))
    sub = [conts[i] for i in sorted(set(min(int(nxt() * len(conts)), len(conts) - 1) for _ in range(k)))]
    for q in covariance_queries(sub):
        if len(qs) < budget:
            qs.append(q)
    # grouped sums and pairwise counts
    for c in cats:
        if len(qs) >= budget:
            break
        if nxt() < 0.6:
            x = conts[min(int(nxt() * len(conts)), len(conts) - 1)]
            qs.append(Query(groupby=[GroupBy(c)], aggs=[Agg.monomial(x)]))
    for i in range(len(cats)):
        for jj in range(i + 1, len(cats)):
            if len(qs) < budget and nxt() < 0.3:
                qs.append(Query(groupby=[GroupBy(cats[i]), GroupBy(cats[jj])]))
    # a few filtered sums
    for _ in range(min(int(nxt() * 6), 5)):
        x = conts[min(int(nxt() * len(conts)), len(conts) - 1)]
        y = conts[min(int(nxt() * len(conts)), len(conts) - 1)]
        qs.append(Query(where=[Pred(x, "le" if nxt() < 0.5 else "gt", float(np.float32(2 * nxt() - 1)))],
                        aggs=[Agg.monomial(y)]))
    return db, qs


def random_covariance_workload(j: int, max_rows: int = 100_000_000, min_rows: int = 1_000_000):
    """Random covariance-only batch number j (seed 9000 + j): a star of a fact
    and 1-4 dimensions, fact rows log-uniform in [min_rows, max_rows],
    dimension rows log-uniform in [100, min(fact / 10, 2M)], 1-20 continuous
    fact attributes and 1-8 per dimension (at most 63 features, so the whole
    batch is one dedicated covariance scan), foreign keys uniform or Zipf(1.2);
    the batch is every covariance entry over all continuous attributes."""
    seed = 9000 + j
    g = native()
    u = g.unit(g.key(seed, "shape"), 256)
    pos = [0]

    def nxt():
        pos[0] += 1
        return float(u[pos[0] - 1])

    def loguni(lo, hi):
        return int(round(math.exp(math.log(lo) + nxt() * (math.log(hi) - math.log(lo)))))

    n_fact = loguni(min_rows, max_rows)
    n_dims = 1 + min(int(nxt() * 4), 3)
    budget = 63
    n_fc = 1 + min(int(nxt() * 20), 19)
    budget -= n_fc
    dims = []
    for i in range(n_dims):
        n_dc = max(1, min(1 + min(int(nxt() * 8), 7), budget - (n_dims - 1 - i)))
        budget -= n_dc
        rows = loguni(100, max(101, min(n_fact // 10, 2_000_000)))
        dims.append(RelSpec("D%d" % (i + 1), rows,
                            [AttrSpec("d%d_%d" % (i + 1, a), "cont", ("normal", 100.0, 1.0)) for a in range(n_dc)],
                            key="k%d" % (i + 1)))
    zipf = {D.key: 1.2 for D in dims if nxt() < 0.6}
    fact = RelSpec("F", n_fact, [AttrSpec("f%d" % a, "cont", ("normal", 100.0, 1.0)) for a in range(n_fc)],
                   children=[(D, D.key) for D in dims], zipf_s=zipf)
    db = build_database(seed, fact)
    return db, covariance_queries(cont_attrs(db))
