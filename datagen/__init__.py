"""Seeded synthetic relations and aggregate batches (inputs only)."""
from .schema import Agg, Column, Database, GroupBy, Pred, Query, Relation  # noqa: F401
from .configs import make_batch, make_database, FULL, SMALL  # noqa: F401
