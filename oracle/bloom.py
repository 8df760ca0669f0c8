"""The Bloom filter variant of Algorithm 1's visited set (section 4.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's GPU kernel keeps the visited nodes of each query in a Bloom filter in
shared memory and accepts its false positives: a node that the filter reports as
visited is never scored by stage 1, and the CPU stages can still reach it.  The paper
gives neither the filter size nor its hash functions.  Readings used here (and by the
library's kernel, which implements the same definition on its own):

* 2^b bits and two hash functions, each the top b bits of the 32-bit product
  v * A mod 2^32 (multiplicative hashing, Knuth, TAOCP vol. 3, 6.4) with the odd
  multipliers A_1 = 0x9E3779B1 and A_2 = 0x85EBCA77;
* a node counts as visited when both of its bits are set;
* the nodes of one group (one adjacency row, or up to 64 entry points) are all
  tested against the filter as it was before the group, then the bits of the fresh
  ones are set; a node listed twice in one group is scored twice and enters C once.
"""

from __future__ import annotations

MULTIPLIERS = (0x9E3779B1, 0x85EBCA77)
ENTRY_GROUP = 64


class BloomFilter:
    """A set of bit positions in [0, 2^log2_bits) with the test and insert above."""

    def __init__(self, log2_bits: int):
        if not 1 <= log2_bits <= 32:
            raise ValueError("log2_bits must be in [1, 32]")
        self.log2_bits = int(log2_bits)
        self.bits_set: set[int] = set()

    def bits(self, v: int) -> tuple[int, int]:
        shift = 32 - self.log2_bits
        return tuple(((int(v) * a) & 0xFFFFFFFF) >> shift for a in MULTIPLIERS)

    def seen(self, v: int) -> bool:
        return all(b in self.bits_set for b in self.bits(v))

    def add(self, v: int) -> None:
        self.bits_set.update(self.bits(v))

    def fresh_of_group(self, group) -> list[int]:
        """The ids of one group to score (in order, repeats kept), then marks them."""
        fresh = [int(v) for v in group if int(v) >= 0 and not self.seen(int(v))]
        for v in fresh:
            self.add(v)
        return fresh
