"""Plain data model for a database, its join tree and an aggregate batch.

The query form is the paper's (Section 1.1 problem statement and the compact
form of Section 2, equation (1)):

    Q(F_1..F_f; alpha_1..alpha_l) += R_1, ..., R_m

* the body is the natural join of all relations (equal attribute names join);
* ``groupby`` lists F: a categorical attribute (cell = its code) or a
  continuous attribute with sorted thresholds t_0 < ... < t_{T-1} (cell =
  bucket = #{k : t_k < x}, so x <= t_k  <=>  bucket <= k);
* ``where`` is a product of Kronecker-delta factors 1[X op t] (Section 1.1);
  a query's aggregates are summed only over join tuples where all hold;
* each aggregate alpha_i = sum_j c_j * prod_k X_jk is a sum of products of
  identity functions of continuous attributes (the empty product is the
  constant 1); COUNT is reported for every cell of every query.

Results are dense over the product of the group-by domains, first group-by
most significant; a cell no tuple reaches has count 0 and sums 0.

This module holds no evaluation arithmetic; it is shared by the oracle, the
engine binding, the tests and the benchmark only as a description of inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

OPS = ("le", "lt", "ge", "gt", "eq", "ne")


@dataclass
class Column:
    attr: str
    kind: str                 # "key" | "key_many" | "cont" | "cat"
    data: np.ndarray          # int32 (key, key_many, cat) or float32 (cont)
    domain: int = 0           # cat: codes in [0, domain); key, key_many: values in [0, domain)
    # "key_many": the join attribute of a child relation whose values may repeat
    # (a many-to-many join)


@dataclass
class Relation:
    name: str
    columns: List[Column]

    @property
    def n_rows(self) -> int:
        return int(len(self.columns[0].data)) if self.columns else 0

    def col(self, attr: str) -> Column:
        for c in self.columns:
            if c.attr == attr:
                return c
        raise KeyError(attr)

    def has(self, attr: str) -> bool:
        return any(c.attr == attr for c in self.columns)


@dataclass
class Database:
    relations: List[Relation]
    edges: List[Tuple[int, int]]          # join tree edges (parent index, child index)

    def rel(self, name: str) -> Relation:
        for r in self.relations:
            if r.name == name:
                return r
        raise KeyError(name)

    def index(self, name: str) -> int:
        for i, r in enumerate(self.relations):
            if r.name == name:
                return i
        raise KeyError(name)

    def owner(self, attr: str) -> int:
        """Index of the one relation that holds a non-key attribute."""
        hits = [i for i, r in enumerate(self.relations) if r.has(attr)]
        if len(hits) != 1:
            raise KeyError("attribute %s held by %d relations" % (attr, len(hits)))
        return hits[0]

    def column(self, attr: str) -> Column:
        """The column of an attribute (for a join key shared by several
        relations, the first holder's column; join tuples agree on it)."""
        for r in self.relations:
            if r.has(attr):
                return r.col(attr)
        raise KeyError(attr)


@dataclass
class GroupBy:
    attr: str
    thresholds: Optional[np.ndarray] = None      # float32, strictly increasing

    def domain(self, db: Database) -> int:
        if self.thresholds is not None:
            return int(len(self.thresholds)) + 1
        return int(db.column(self.attr).domain)


@dataclass
class Pred:
    attr: str
    op: str
    value: float


@dataclass
class Agg:
    terms: List[Tuple[float, Tuple[str, ...]]]    # sum of coeff * product of attrs

    @staticmethod
    def monomial(*attrs: str) -> "Agg":
        return Agg([(1.0, tuple(attrs))])


@dataclass
class Query:
    groupby: List[GroupBy] = field(default_factory=list)
    where: List[Pred] = field(default_factory=list)
    aggs: List[Agg] = field(default_factory=list)

    def n_cells(self, db: Database) -> int:
        n = 1
        for g in self.groupby:
            n *= g.domain(db)
        return n


def count_query() -> Query:
    return Query()


def sum_query(*attrs: str, groupby: Sequence[GroupBy] = (), where: Sequence[Pred] = ()) -> Query:
    return Query(list(groupby), list(where), [Agg.monomial(*attrs)])
