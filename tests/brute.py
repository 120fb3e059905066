"""String-level brute-force k-mer counter used to pin the oracle.

It never packs bases into integers: a k-mer is a Python string, its reverse
complement is built character by character, the canonical form is the smaller
string, and occurrences go into a dict.  Sorting the strings gives the reference
order (A < C < G < T in ASCII).
"""
from typing import Dict, Iterable, List, Tuple

_COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}
_VALID = set("ACGTacgt")


def brute_count(seqs: Iterable[str], k: int) -> Dict[str, int]:
    d: Dict[str, int] = {}
    for s in seqs:
        for i in range(len(s) - k + 1):
            w = s[i:i + k]
            if not all(ch in _VALID for ch in w):
                continue
            w = w.upper()
            rc = "".join(_COMP[ch] for ch in reversed(w))
            c = w if w <= rc else rc
            d[c] = d.get(c, 0) + 1
    return d


def brute_occurrences(seqs: Iterable[str], k: int) -> Dict[str, List[Tuple[int, int]]]:
    """Canonical k-mer string -> list of (read index, window start), in read order."""
    d: Dict[str, List[Tuple[int, int]]] = {}
    for r, s in enumerate(seqs):
        for i in range(len(s) - k + 1):
            w = s[i:i + k]
            if not all(ch in _VALID for ch in w):
                continue
            w = w.upper()
            rc = "".join(_COMP[ch] for ch in reversed(w))
            d.setdefault(w if w <= rc else rc, []).append((r, i))
    return d


def canonical_str(w: str) -> str:
    w = w.upper()
    rc = "".join(_COMP[ch] for ch in reversed(w))
    return w if w <= rc else rc


def decode(words, k: int) -> str:
    """Integer k-mer (first base in the most significant two bits) -> string."""
    v = int(words[0])
    if len(words) > 1:
        v |= int(words[1]) << 64
    return "".join("ACGT"[(v >> (2 * (k - 1 - j))) & 3] for j in range(k))


def split_reads(reads, offsets) -> List[str]:
    raw = bytes(reads)
    return [raw[int(offsets[i]):int(offsets[i + 1])].decode("latin-1") for i in range(len(offsets) - 1)]


def pairs_of(res, k: int) -> List[Tuple[str, int]]:
    return [(decode(res.kmers[i], k), int(res.counts[i])) for i in range(res.n_pairs)]


def de_bruijn(n: int, alphabet: int = 4) -> List[int]:
    """Lexicographically least de Bruijn sequence B(alphabet, n) (cyclic), from the
    Lyndon words whose length divides n, generated in order (Fredricksen-Kessler-
    Maiorana, with Duval's successor rule)."""
    seq: List[int] = []
    w = [-1]
    while w:
        w[-1] += 1
        m = len(w)
        if n % m == 0:
            seq.extend(w)
        while len(w) < n:
            w.append(w[len(w) - m])
        while w and w[-1] == alphabet - 1:
            w.pop()
    return seq
