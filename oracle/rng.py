"""SplitMix64, the counter-based generator used to draw sample positions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper asks for a random sample (Section 6) without fixing a generator.
Both the oracle and the GPU library implement SplitMix64 independently from
its published definition (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the state advances by the
golden gamma 0x9E3779B97F4A7C15 and each output is the state passed through
the mixing function ``mix64`` below.  The i-th output (i >= 1) of a generator
started at state s is therefore mix64(s + i * gamma), a pure function of
(s, i).

Pin: ``tests/golden/splitmix64.txt`` holds the generator's published first
outputs for seeds 0 and 1234567.  ``stream_state`` is a convention of this
project (the paper fixes no generator); its first fold is the published
first output at the seed, distinct (level, root, offset) keys give distinct
states, and ``sample_positions`` for n = 2^k is the top k bits of the
published stream, uniform by a chi-square test.
"""

from __future__ import annotations

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    """SplitMix64 output function (variant 13 of Stafford's mixers)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64_outputs(seed: int, count: int) -> list:
    """First ``count`` outputs of SplitMix64 started at state ``seed``."""
    return [mix64(seed + i * GAMMA) for i in range(1, count + 1)]


def stream_state(seed: int, level: int, root: int, offset: int) -> int:
    """Generator state for one subproblem: seed, level (0-based), root index
    and the subproblem's offset inside its root, folded in with mix64."""
    s = mix64((seed + GAMMA) & M64)
    s = mix64(s ^ (level + 1))
    s = mix64(s ^ root)
    s = mix64(s ^ offset)
    return s


def sample_positions(seed: int, level: int, root: int, offset: int, n: int, count: int) -> list:
    """``count`` uniform positions in [0, n), drawn with replacement.

    Position i is floor(n * u_i / 2^64) where u_i is output i+1 of the
    generator at ``stream_state(...)``.
    """
    s = stream_state(seed, level, root, offset)
    return [(mix64((s + (i + 1) * GAMMA) & M64) * n) >> 64 for i in range(count)]
