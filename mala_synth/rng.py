"""SplitMix64 counter-free stream generator and the draws built on it.

SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the output is
mixed with two xor-shift-multiply rounds.  Uniforms take the top 53 bits;
normals use the Box-Muller transform.  Everything here is vectorised with
numpy uint64 arithmetic (wrap-around multiply is the intended semantics).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


class SplitMix64:
    """Sequential SplitMix64 stream; draws of size n advance the state by n."""

    def __init__(self, seed):
        self.state = np.uint64(int(seed) & 0xFFFFFFFFFFFFFFFF)

    def next_u64(self, n):
        with np.errstate(over="ignore"):
            steps = np.arange(1, n + 1, dtype=np.uint64)
            z = self.state + steps * _GOLDEN
            self.state = self.state + np.uint64(n) * _GOLDEN
            return _mix(z)

    def uniform(self, n):
        """n doubles in [0, 1) from the top 53 bits."""
        return (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def uniform_range(self, n, lo, hi):
        return lo + (hi - lo) * self.uniform(n)

    def normal(self, n):
        """n standard normals by Box-Muller (pairs; first uniform kept off 0)."""
        m = (n + 1) // 2
        u1 = 1.0 - self.uniform(m)          # (0, 1]
        u2 = self.uniform(m)
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.empty(2 * m)
        z[0::2] = r * np.cos(2.0 * np.pi * u2)
        z[1::2] = r * np.sin(2.0 * np.pi * u2)
        return z[:n]
