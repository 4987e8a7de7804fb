"""Seeded synthetic protein-family workloads.

This module only draws random sequences.  It holds none of the similarity
arithmetic, so both the GPU path and the CPU oracle may take their inputs from
it without sharing any of the method.

Sequences are uint8 codes over a 20-letter amino-acid alphabet (the paper's
Methods section, "Progressive construction of the alignment", fixes the
alphabet at 32 codes: twenty amino acids plus special symbols; the synthetic
families use codes 0..19 only).

A workload is a ``Batch``: every sequence concatenated into one ``codes``
array, ``seq_off`` (nseq + 1 offsets into it) and ``fam_off`` (nfam + 1
offsets into the sequence list).  Pairs are only formed inside a family.

The five named workloads (the paper has no public data for this stage, so
these stand in for its large protein families):

* ``c1``: 100 i.i.d. sequences, lengths uniform in [50, 300], seed 0.
* ``c2``: one tree-evolved family, k = 10,000, root length 300, seed 1.
* ``c3``: 64 tree-evolved families, k log-uniform in [50, 5000], root
  length log-uniform in [30, 2000], seed 2.
* ``c4``: one tree-evolved family, k = 100,000, root length 250, each leaf
  trimmed or padded to a log-normal target length (median 250, sigma 0.3,
  clipped to [40, 1500]), seed 3.
* ``c5``: serving jobs, each a tree-evolved family with k log-uniform in
  [100, 20000] and root length log-uniform in [50, 1500], Poisson arrivals,
  seed 4.

Tree evolution: a random binary tree made by recursive uniform splitting (a
node over n leaves sends U{1..n-1} leaves left); along every edge each residue
is substituted with probability 0.10 by a uniformly chosen different residue,
then indel events occur at 0.02 per residue, half insertions and half
deletions, each of Geometric(0.5) length on {1, 2, ...}; inserted residues
are i.i.d. uniform; a sequence never shrinks below one residue.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ALPHABET = 20          # codes 0..19 in every synthetic workload
GENERATOR_VERSION = 1  # bump when any recipe below changes

SUB_RATE = 0.10
INDEL_RATE = 0.02
INDEL_GEOM_P = 0.5


@dataclasses.dataclass
class Batch:
    """Concatenated sequences grouped into families."""
    codes: np.ndarray      # uint8, all residues back to back
    seq_off: np.ndarray    # uint64, nseq + 1
    fam_off: np.ndarray    # uint32, nfam + 1
    name: str = ""
    seed: int = 0

    @property
    def nseq(self) -> int:
        return int(self.seq_off.shape[0] - 1)

    @property
    def nfam(self) -> int:
        return int(self.fam_off.shape[0] - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.seq_off).astype(np.int64)

    def family(self, f: int) -> "Batch":
        a, b = int(self.fam_off[f]), int(self.fam_off[f + 1])
        lo, hi = int(self.seq_off[a]), int(self.seq_off[b])
        return Batch(self.codes[lo:hi].copy(), (self.seq_off[a:b + 1] - lo).astype(np.uint64),
                     np.array([0, b - a], dtype=np.uint32), f"{self.name}[{f}]", self.seed)

    def seq(self, i: int) -> np.ndarray:
        return self.codes[int(self.seq_off[i]):int(self.seq_off[i + 1])]

    def family_sizes(self) -> np.ndarray:
        return np.diff(self.fam_off).astype(np.int64)

    def pairs(self) -> int:
        k = self.family_sizes()
        return int(np.sum(k * (k - 1) // 2))

    def cells(self) -> int:
        """Sum over in-family pairs i<j of |A_i|*|A_j| (exact, int)."""
        L = self.lengths()
        tot = 0
        for f in range(self.nfam):
            a, b = int(self.fam_off[f]), int(self.fam_off[f + 1])
            s = int(L[a:b].sum())
            sq = int((L[a:b] * L[a:b]).sum())
            tot += (s * s - sq) // 2
        return tot


def from_sequences(seqs: Sequence[np.ndarray], families: Optional[Sequence[int]] = None,
                   name: str = "", seed: int = 0) -> Batch:
    """Build a Batch from a list of code arrays; ``families`` gives family sizes."""
    seqs = [np.asarray(s, dtype=np.uint8) for s in seqs]
    lens = np.array([len(s) for s in seqs], dtype=np.uint64)
    off = np.zeros(len(seqs) + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    codes = np.concatenate(seqs) if len(seqs) and int(off[-1]) > 0 else np.zeros(0, np.uint8)
    if families is None:
        families = [len(seqs)]
    fam = np.zeros(len(families) + 1, dtype=np.uint32)
    np.cumsum(np.asarray(families, dtype=np.uint32), out=fam[1:])
    assert int(fam[-1]) == len(seqs)
    return Batch(codes.astype(np.uint8), off, fam, name, seed)


# ---------------------------------------------------------------- evolution

def _mutate(seq: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """One tree edge: substitutions, then insertions/deletions."""
    L = seq.shape[0]
    out = seq.copy()
    if L:
        hit = rng.random(L) < SUB_RATE
        nh = int(hit.sum())
        if nh:
            out[hit] = (out[hit].astype(np.int16) + rng.integers(1, ALPHABET, nh)) % ALPHABET
    nev = int(rng.binomial(L, INDEL_RATE)) if L else 0
    if nev == 0:
        return out
    pos = np.sort(rng.integers(0, L + 1, nev))
    ins = rng.random(nev) < 0.5
    ln = rng.geometric(INDEL_GEOM_P, nev)
    pieces: List[np.ndarray] = []
    cur = 0
    for p, is_ins, n in zip(pos.tolist(), ins.tolist(), ln.tolist()):
        if p < cur:          # inside a region an earlier deletion removed
            p = cur
        pieces.append(out[cur:p])
        if is_ins:
            pieces.append(rng.integers(0, ALPHABET, n).astype(np.uint8))
            cur = p
        else:
            cur = min(L, p + n)
    pieces.append(out[cur:])
    res = np.concatenate(pieces).astype(np.uint8)
    if res.shape[0] == 0:
        res = rng.integers(0, ALPHABET, 1).astype(np.uint8)
    return res


def evolve_family(k: int, root_len: int, rng: np.random.Generator) -> List[np.ndarray]:
    """k leaves of a random binary tree grown from a random root."""
    root = rng.integers(0, ALPHABET, root_len).astype(np.uint8)
    leaves: List[np.ndarray] = []
    stack = [(root, k)]
    while stack:
        s, n = stack.pop()
        if n == 1:
            leaves.append(s)
            continue
        nl = int(rng.integers(1, n))
        # push right first so leaves come out left to right
        stack.append((_mutate(s, rng), n - nl))
        stack.append((_mutate(s, rng), nl))
    return leaves


def _log_uniform_int(rng: np.random.Generator, lo: float, hi: float) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


# ---------------------------------------------------------------- workloads

def c1(seed: int = 0, k: int = 100, lo: int = 50, hi: int = 300) -> Batch:
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, k)
    seqs = [rng.integers(0, ALPHABET, int(n)).astype(np.uint8) for n in lens]
    return from_sequences(seqs, name="c1", seed=seed)


def c2(seed: int = 1, k: int = 10_000, root_len: int = 300) -> Batch:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    return from_sequences(evolve_family(k, root_len, rng), name="c2", seed=seed)


def c3(seed: int = 2, nfam: int = 64, k_range=(50, 5000), root_range=(30, 2000)) -> Batch:
    ss = np.random.SeedSequence(seed).spawn(nfam)
    seqs: List[np.ndarray] = []
    sizes: List[int] = []
    for f in range(nfam):
        rng = np.random.default_rng(ss[f])
        k = _log_uniform_int(rng, *k_range)
        L = _log_uniform_int(rng, *root_range)
        seqs += evolve_family(k, L, rng)
        sizes.append(k)
    return from_sequences(seqs, sizes, name="c3", seed=seed)


def c4(seed: int = 3, k: int = 100_000, root_len: int = 250, sigma: float = 0.3,
       clip=(40, 1500)) -> Batch:
    s_tree, s_len = np.random.SeedSequence(seed).spawn(2)
    rng = np.random.default_rng(s_tree)
    leaves = evolve_family(k, root_len, rng)
    lr = np.random.default_rng(s_len)
    target = np.clip(np.round(root_len * np.exp(sigma * lr.standard_normal(k))), clip[0], clip[1]).astype(np.int64)
    out = []
    for s, T in zip(leaves, target.tolist()):
        if s.shape[0] >= T:
            out.append(s[:T])
        else:
            out.append(np.concatenate([s, lr.integers(0, ALPHABET, T - s.shape[0]).astype(np.uint8)]))
    return from_sequences(out, name="c4", seed=seed)


@dataclasses.dataclass
class ServeJob:
    arrival_s: float
    batch: Batch


def _c5_job(args) -> Batch:
    j, ss, k_range, root_range, k_scale, seed = args
    rng = np.random.default_rng(ss)
    k = _log_uniform_int(rng, *k_range)
    L = _log_uniform_int(rng, *root_range)
    k = max(2, int(round(k * k_scale)))
    return from_sequences(evolve_family(k, L, rng), name=f"c5job{j}", seed=seed)


def c5(seed: int = 4, njobs: int = 200, rate_per_s: float = 2.0, k_range=(100, 20000),
       root_range=(50, 1500), k_scale: float = 1.0, workers: int = 0) -> List[ServeJob]:
    """Serving jobs with Poisson arrivals at ``rate_per_s`` jobs per second.

    ``k_scale`` shrinks every family size (k -> max(2, round(k * k_scale)))
    so the same arrival stream can be replayed at a smaller cost.  Each job
    draws from its own spawned seed, so ``workers`` > 1 (processes building
    jobs in parallel) gives the same jobs.
    """
    root = np.random.SeedSequence(seed)
    s_arr, s_jobs = root.spawn(2)
    arr = np.cumsum(np.random.default_rng(s_arr).exponential(1.0 / rate_per_s, njobs))
    args = [(j, ss, k_range, root_range, k_scale, seed) for j, ss in enumerate(s_jobs.spawn(njobs))]
    if workers > 1 and njobs > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, njobs)) as pool:
            batches = pool.map(_c5_job, args, chunksize=1)
    else:
        batches = [_c5_job(a) for a in args]
    return [ServeJob(float(arr[j]), b) for j, b in enumerate(batches)]


def random_family(k: int, lo: int, hi: int, seed: int, alphabet: int = ALPHABET) -> Batch:
    """i.i.d. family with lengths uniform in [lo, hi] (edge and parity cases)."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, k)
    return from_sequences([rng.integers(0, alphabet, int(n)).astype(np.uint8) for n in lens],
                          name=f"rand{k}_{lo}_{hi}", seed=seed)


def stats(b: Batch) -> dict:
    L = b.lengths()
    return {"name": b.name, "seed": b.seed, "nseq": b.nseq, "nfam": b.nfam,
            "pairs": b.pairs(), "cells": b.cells(),
            "len_mean": float(L.mean()) if L.size else 0.0,
            "len_sd": float(L.std()) if L.size else 0.0,
            "len_min": int(L.min()) if L.size else 0, "len_max": int(L.max()) if L.size else 0,
            "generator_version": GENERATOR_VERSION}


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4}


# ---------------------------------------------------------------- profiles

GAP = 0xFF  # a gap in a gapped profile row


@dataclasses.dataclass
class ProfileProblem:
    """One sequence to align to a profile of K gapped rows of width n."""
    seq: np.ndarray    # uint8, m codes
    rows: np.ndarray   # uint8, K x n, codes or GAP


def synthetic_subst(sigma: int, seed: int) -> np.ndarray:
    """A symmetric integer substitution matrix (sigma x sigma, int32): the
    diagonal uniform in [4, 12], the rest uniform in [-4, 2].  The paper
    names MIQS but does not print its values, so a synthetic matrix of that
    shape stands in for it."""
    rng = np.random.default_rng(seed)
    S = rng.integers(-4, 3, (sigma, sigma))
    S = np.triu(S) + np.triu(S, 1).T
    S[np.arange(sigma), np.arange(sigma)] = rng.integers(4, 13, sigma)
    return S.astype(np.int32)


def profile_problem(m_target: int, n: int, K: int, rng: np.random.Generator, alphabet: int = ALPHABET,
                    p_conserved: float = 0.7, p_open: float = 0.05, p_terminal: float = 0.3,
                    p_empty_row: float = 0.0) -> ProfileProblem:
    """A profile whose columns are noisy copies of a random consensus, and a
    sequence drawn near the same consensus.

    Each row: with probability ``p_terminal`` a leading and (independently) a
    trailing gap run of uniform length up to n/4; inside, gap runs open with
    probability ``p_open`` per column and have Geometric(1/3) lengths; every
    other column holds the consensus symbol with probability ``p_conserved``,
    else a uniform one.  With probability ``p_empty_row`` a row is all gaps.
    The sequence: the consensus resampled to ``m_target`` positions (drop or
    repeat evenly), 10% of residues substituted.
    """
    cons = rng.integers(0, alphabet, max(n, 1)).astype(np.uint8)
    rows = np.full((K, n), GAP, dtype=np.uint8)
    for s in range(K):
        if n == 0 or rng.random() < p_empty_row:
            continue
        lead = int(rng.integers(0, n // 4 + 1)) if rng.random() < p_terminal else 0
        trail = int(rng.integers(0, n // 4 + 1)) if rng.random() < p_terminal else 0
        c = lead
        while c < n - trail:
            if rng.random() < p_open:
                c += int(rng.geometric(1.0 / 3.0))
                continue
            rows[s, c] = cons[c] if rng.random() < p_conserved else rng.integers(0, alphabet)
            c += 1
    if m_target <= 0:
        seq = np.zeros(0, np.uint8)
    else:
        idx = np.minimum((np.arange(m_target) * max(n, 1)) // m_target, max(n, 1) - 1)
        seq = cons[idx].copy()
        hit = rng.random(m_target) < 0.1
        seq[hit] = rng.integers(0, alphabet, int(hit.sum()))
    return ProfileProblem(seq.astype(np.uint8), rows)


def profile_batch(nprob: int, seed: int, m_range=(50, 400), K_range=(1, 200), alphabet: int = ALPHABET):
    """A progressive-stage level: ``nprob`` independent problems, profile
    width log-uniform in ``m_range``, the sequence within +-15% of it, and
    K log-uniform in ``K_range``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nprob):
        n = _log_uniform_int(rng, *m_range)
        m = max(1, int(round(n * rng.uniform(0.85, 1.15))))
        K = _log_uniform_int(rng, *K_range)
        out.append(profile_problem(m, n, K, rng, alphabet))
    return out
