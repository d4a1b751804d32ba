"""Counter-based Gaussian random test matrices for peeling (oracle side).

The paper samples with "random vectors" (Sec. 3.3, block sampling); the
workloads fix seeded N(0,1) entries.  Both the oracle and the HIP library
implement the same published generator independently so that the same
Omega is drawn on both sides:

  splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): the n-th output of the stream whose state starts
  at `key` is  mix64(key + n * GAMMA)  for n = 1, 2, ...,  with
      mix64(z): z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
                z = (z ^ (z >> 27)) * 0x94D049BB133111EB
                return z ^ (z >> 31)            (all mod 2^64)

  Key of a stream: key = mix64(mix64(seed + GAMMA) ^ tag), with
      tag = phase << 56 | level << 48 | round << 32 | iteration  (bit fields).
  Entry (row r in tree order, column j) uses outputs n = 2*(r*2^16 + j) + 1
  and n + 1, mapped to uniforms u = ((x >> 11) + 1) * 2^-53 in (0, 1], and the
  Box-Muller transform z = sqrt(-2 ln u1) * cos(2 pi u2).
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)

# phases of the method that draw random matrices
PHASE_NORM = 1     # power-iteration start vectors
PHASE_RANGE = 2    # range-finder samples of peeling
PHASE_PROBE = 5    # independent error probes (tests)
PHASE_RESID = 6    # power iteration on the Newton-Schulz residual


def mix64(z):
    """splitmix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(state, count):
    """First `count` outputs of splitmix64 started at `state` (reference form)."""
    n = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(state) + n * GAMMA)


def stream_key(seed, phase, level, rnd, iteration=0):
    tag = (np.uint64(phase) << np.uint64(56)) | (np.uint64(level) << np.uint64(48)) \
        | (np.uint64(rnd) << np.uint64(32)) | np.uint64(iteration)
    with np.errstate(over="ignore"):
        return mix64(mix64(np.uint64(seed) + GAMMA) ^ tag)


def gaussian(key, rows, cols):
    """Gaussian block for the given tree-order rows (array) and columns (array).

    Returns an array of shape (len(rows), len(cols)) in float64.
    """
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, 1)
    cols = np.asarray(cols, dtype=np.uint64).reshape(1, -1)
    with np.errstate(over="ignore"):
        n = np.uint64(2) * ((rows << np.uint64(16)) + cols) + np.uint64(1)
        x1 = mix64(np.uint64(key) + n * GAMMA)
        x2 = mix64(np.uint64(key) + (n + np.uint64(1)) * GAMMA)
    scale = 2.0 ** -53
    u1 = ((x1 >> np.uint64(11)).astype(np.float64) + 1.0) * scale
    u2 = ((x2 >> np.uint64(11)).astype(np.float64) + 1.0) * scale
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
