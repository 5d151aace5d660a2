"""SplitMix64, written from its published definition.

Steele, Lea and Flood, "Fast Splittable Pseudorandom Number Generators",
OOPSLA 2014: the state advances by the odd constant 0x9E3779B97F4A7C15 and each
output is the state passed through the 64-bit variant-13 finaliser
(xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31).

The array-code search draws its random numbers from this generator; the HIP
library implements the same published generator on its own side.

Pin: the first outputs for seed 0 are the published test vector
(tests/test_oracle_codes.py).
"""

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


class SplitMix64:
    """Sequential SplitMix64 stream seeded with a 64-bit integer."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * _M1) & _MASK
        z = ((z ^ (z >> 27)) * _M2) & _MASK
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        """A draw in [0, n) taken as the plain remainder of one output."""
        return self.next() % n
