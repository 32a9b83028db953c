"""Seeded synthetic workloads: face-template databases and queries.

This module is shared by the HIP path, the oracle-side tests and the
benchmark.  It draws inputs only -- it holds none of the encryption method's
arithmetic and imports nothing else from the package.

Stand-in for the paper's data (§6.1, "Datasets"): the FRGC 2.0 embeddings and
the ArcFace extractor are not available, so templates are 512-d (or 128-d)
unit vectors.  Non-matching templates are i.i.d. standard Gaussian rows
normalised to unit L2 norm; a planted template has cosine c ~ U[0.6, 0.9] to
the query: t = c x + sqrt(1 - c^2) u, with u a unit Gaussian vector
orthogonalised against x.  Positions of the planted templates are uniform
without replacement.  Everything is stored as float32 after normalisation.

Seeds: master seed 0x5EED0000 + config, with numbered sub-streams
(1 database, 2 query, 3 planted positions and cosines, 4 key material,
6 encryption, 7 batch sizes, 8 arrivals, 9 request types).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MASTER = 0x5EED0000

SUB_DB, SUB_QUERY, SUB_PLANT, SUB_KEYS, SUB_ENC, SUB_BATCH, SUB_ARRIVAL, SUB_KIND = 1, 2, 3, 4, 6, 7, 8, 9


def rng(config: int, sub: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([MASTER + config, sub, extra])))


def int_seed(config: int, sub: int, extra: int = 0) -> int:
    """A 64-bit integer seed for the counter-based generator of key material
    or of an encryption."""
    return int(rng(config, sub, extra).integers(0, 2**63, dtype=np.int64))


def unit_rows(g: np.random.Generator, n: int, d: int) -> np.ndarray:
    x = g.standard_normal((n, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


@dataclass
class Workload:
    templates: np.ndarray          # [K][ell] float32, unit rows
    query: np.ndarray              # [ell] float32, unit
    planted: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    cosines: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def K(self) -> int:
        return self.templates.shape[0]

    @property
    def ell(self) -> int:
        return self.templates.shape[1]

    def exact_scores(self) -> np.ndarray:
        """FP64 inner products of every template with the query."""
        return self.templates.astype(np.float64) @ self.query.astype(np.float64)


def make_workload(config: int, K: int, ell: int, planted_frac: float = 0.0, extra: int = 0) -> Workload:
    T = unit_rows(rng(config, SUB_DB, extra), K, ell)
    x = unit_rows(rng(config, SUB_QUERY, extra), 1, ell)[0]
    planted = np.zeros(0, dtype=np.int64)
    cos = np.zeros(0)
    n_plant = int(round(planted_frac * K))
    if n_plant:
        g = rng(config, SUB_PLANT, extra)
        planted = np.sort(g.choice(K, size=n_plant, replace=False)).astype(np.int64)
        cos = g.uniform(0.6, 0.9, size=n_plant)
        xd = x.astype(np.float64)
        u = g.standard_normal((n_plant, ell))
        u -= np.outer(u @ xd, xd) / (xd @ xd)
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        t = cos[:, None] * xd[None, :] + np.sqrt(1.0 - cos ** 2)[:, None] * u
        t /= np.linalg.norm(t, axis=1, keepdims=True)
        T[planted] = t.astype(np.float32)
    return Workload(T, x, planted, cos)


def replicate_query(x: np.ndarray, n_slots: int) -> np.ndarray:
    """Slot vector carrying n_slots / ell copies of the query (period ell)."""
    ell = len(x)
    return np.tile(x.astype(np.float64), n_slots // ell)


def query_batch(config: int, nq: int, ell: int) -> np.ndarray:
    """nq unit-norm queries (float32 rows), query q drawn from its own stream."""
    return np.stack([unit_rows(rng(config, SUB_QUERY, 1 + q), 1, ell)[0] for q in range(nq)])
