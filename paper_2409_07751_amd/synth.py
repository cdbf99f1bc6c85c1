"""Seeded synthetic workloads: parameter sizes, KAN shapes, random weights and
inputs.  This module holds none of the method's arithmetic; it only draws
numbers, so both the GPU path and the CPU checker can take their inputs from
it.

Workloads (the data sets of the paper are not available; these inputs have
their shapes and value ranges):
  tiny    N=2^13, 8 Q primes (60 + 7x40 bits), 1 special prime, scale 2^40,
          KAN [2,5,1], k=3, G=5 on [-1,1], c ~ N(0, 0.1^2), w_b ~ N(0, 0.3^2),
          SiLU degree 15 on [-4,4], one input x ~ U[-1,1]^2;
  formula N=2^15, 17 Q primes (60 + 16x40), 2 special primes, scale 2^40,
          KAN [4,10,10,1], k=3, G=10 on [-1,1], SiLU degree 27 (data range);
  image   N=2^16, 25 Q primes (60 + 24x45), 4 special primes, scale 2^45,
          KAN [784,64,10], k=3, G=8 on [0,1], weights N(0, 0.05^2), SiLU
          degree 31, 28x28 images with pixels U[0,1] quantised to k/255
          (the MNIST shape), raster-scanned;
  cifar   same parameters, KAN [3072,128,10] on 32x32x3 images (the CIFAR-10
          shape), pixels U[0,1];
  toy     the tiny parameters, KAN [2,3,1] with g=2, k=1 (the grid of the
          paper's toy example of the basis construction);
  tiny16  the tiny KAN [2,5,1] at the image parameters (uneven-shape mix);
  tinydeep the tiny KAN with a depth-12 comparison composite, run with
          bootstrapping between layers (boot11deep).
Bootstrappable parameter sets (BOOTSETS) carry their own chains.
Seeds: weights 1, inputs 2, keygen 3, encryption 4, arrivals 5, calibration 6.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_WEIGHTS, SEED_INPUTS, SEED_KEYGEN, SEED_ENC, SEED_ARRIVALS, SEED_CALIB = 1, 2, 3, 4, 5, 6


@dataclass(frozen=True)
class Workload:
    name: str
    logN: int
    L: int
    scale_bits: int
    alpha: int
    w: int                       # key-switch digit width in Q limbs
    shape: tuple                 # KAN layer widths
    g: int
    k: int
    grid: tuple                  # grid of the first layer
    silu_degree: int
    silu_range: tuple = None     # fixed SiLU range, or None for the data range
    comp_degrees: tuple = ()     # comparison composite stage degrees per layer
    wb_std: float = 0.3
    c_std: float = 0.1
    input_kind: str = "uniform_pm1"
    refresh: bool = False        # client-aided refresh between layers
    prescale: bool = True        # explicit 1/(2R) before PolyComp (False: folded, saves a level)
    base_bits: int = 60
    special_bits: int = 60
    sigma: float = 3.2


WORKLOADS = {
    "tiny": Workload("tiny", 13, 7, 40, 1, 1, (2, 5, 1), 5, 3, (-1.0, 1.0), 15, (-4.0, 4.0),
                     ((3,), (3,)), 0.3, 0.1, "uniform_pm1", True, False),
    "formula": Workload("formula", 15, 16, 40, 2, 2, (4, 10, 10, 1), 10, 3, (-1.0, 1.0), 27, None,
                        ((7, 7), (7, 7), (7, 7)), 0.3, 0.1, "uniform_pm1", True),
    # the [4,10,10,1] formula-scale KAN at the image parameters (serving mix):
    # three 8-level layers, f_3 with 1/(2R) folded (R is small on [-1, 1])
    "formula16": Workload("formula16", 16, 24, 45, 4, 5, (4, 10, 10, 1), 10, 3, (-1.0, 1.0), 27, None,
                          ((7,), (7,), (7,)), 0.3, 0.1, "uniform_pm1", False, False),
    # the [2,5,1] tiny KAN at the image parameters (the batched mix of uneven
    # shapes): two 7-level layers fit the 24 levels without a refresh
    "tiny16": Workload("tiny16", 16, 24, 45, 4, 5, (2, 5, 1), 5, 3, (-1.0, 1.0), 15, (-4.0, 4.0),
                       ((3,), (3,)), 0.3, 0.1, "uniform_pm1", False, False),
    "image": Workload("image", 16, 24, 45, 4, 5, (784, 64, 10), 8, 3, (0.0, 1.0), 31, None,
                      ((7, 7), (7, 7)), 0.05, 0.05, "pixels255"),
    "cifar": Workload("cifar", 16, 24, 45, 4, 5, (3072, 128, 10), 8, 3, (0.0, 1.0), 31, None,
                      ((7, 7), (7, 7)), 0.05, 0.05, "pixels"),
    # the paper's toy example of the basis construction (g = 2, k = 1): g+2k = 4
    # repeat-packed copies, one block short of the g+2k+1 a shared second
    # comparison needs, so the first layer runs Algorithm 2 with both PolyComps
    "toy": Workload("toy", 13, 7, 40, 1, 1, (2, 3, 1), 2, 1, (-1.0, 1.0), 15, (-4.0, 4.0),
                    ((3,), (3,)), 0.3, 0.1, "uniform_pm1", True, False),
    # the tiny KAN with a depth-12 comparison composite (f_3 four times, 1/(2R)
    # folded): 17 levels per layer, which the bootstrappable set boot11deep
    # holds between refreshes; its HE-friendly network is within 1e-2 of the
    # exact KAN (the shallow composites of the other workloads are not)
    "tinydeep": Workload("tinydeep", 11, 17, 45, 3, 3, (2, 5, 1), 5, 3, (-1.0, 1.0), 15, (-4.0, 4.0),
                         ((7, 7, 7, 7), (7, 7, 7, 7)), 0.3, 0.1, "uniform_pm1", False, False, 55),
    # the tiny parameters with a first layer too wide for one ciphertext
    # (384 x 16 repeat-packed slots > 4096): two input ciphertexts
    "tinychunk": Workload("tinychunk", 13, 7, 40, 1, 1, (384, 4, 1), 5, 3, (-1.0, 1.0), 15, (-4.0, 4.0),
                          ((3,), (3,)), 0.3, 0.1, "uniform_pm1", True, False),
}


@dataclass(frozen=True)
class BootSet:
    """A bootstrappable parameter set: computation levels 1..Lc with primes
    of scale_bits under boot_levels primes of boot_bits (the levels a
    bootstrapping consumes), a sparse ternary secret of Hamming weight h, and
    the bootstrapping's shape: stage groups (levels) of CoeffToSlot and
    SlotToCoeff, EvalMod's input range [-K, K], r double-angle steps and the
    degree of its cosine series."""
    name: str
    logN: int
    Lc: int
    boot_levels: int
    scale_bits: int
    boot_bits: int
    alpha: int
    w: int
    h: int
    cts: int
    stc: int
    K: float
    r: int
    degree: int
    base_bits: int = 60
    special_bits: int = 60
    sigma: float = 3.2
    real_stc: int = 2  # SlotToCoeff groups of the real-slot refresh (levels it takes from its input)

    @property
    def L(self):
        return self.Lc + self.boot_levels


# boot11: N=2^11, 55 + 8x45 + 14x58 bits, 2 special primes, 2-limb digits,
#   h = 32 (|I| <= 12 holds with margin: std sqrt(33/12) = 1.7); the 8
#   computation levels hold one layer of the [4,10,10,1] formula KAN;
# boot16: N=2^16, 51 + 10x45 + 17x58 bits, 4 special primes, 4-limb digits,
#   h = 192 (|I| <= 32 is 8 standard deviations of sqrt(193/12) = 4.0).
# The base prime's size balances EvalMod's two errors: a smaller q_0 raises
# the message against the rounding in CoeffToSlot (whose slots carry q_0 I),
# a larger one keeps sin(2 pi m/q_0) closer to 2 pi m/q_0 (measured on the
# oracle at |z| <= 1: q_0 of 60 bits 3.4e-5, 55 bits 1.1e-6, 53 bits 3.3e-7,
# 51 bits 1.1e-7 at N=2^16; 60 bits 2.1e-7, 55 bits 9.6e-9, 52 bits 3.2e-7
# at N=2^11)
BOOTSETS = {
    "boot11": BootSet("boot11", 11, 8, 14, 45, 58, 2, 2, 32, 2, 2, 12.0, 4, 23, base_bits=55),
    "boot16": BootSet("boot16", 16, 10, 17, 45, 58, 4, 4, 192, 3, 3, 32.0, 5, 27, base_bits=51),
    # boot11's refresh under 17 computation levels (3 special primes, 3-limb digits)
    "boot11deep": BootSet("boot11deep", 11, 17, 14, 45, 58, 3, 3, 32, 2, 2, 12.0, 4, 23, base_bits=55),
}


def boot_inputs(bs: BootSet, n, stream=0):
    """n real slot vectors (all N/2 slots) with values U[-1, 1]."""
    return _rng(SEED_INPUTS, 100 + stream).uniform(-1.0, 1.0, (n, 1 << (bs.logN - 1)))


def _rng(*key):
    return np.random.default_rng(list(key))


def raw_weights(wl: Workload, seed=SEED_WEIGHTS):
    """Random-init weights of the KAN shape: per layer w_b (n_out x n_in),
    w_s = 1 and per-edge spline coefficients c (n_out x n_in x (g+k))."""
    layers = []
    for li in range(len(wl.shape) - 1):
        n_in, n_out = wl.shape[li], wl.shape[li + 1]
        r = _rng(seed, li)
        wb = r.normal(0.0, wl.wb_std, (n_out, n_in))
        c = r.normal(0.0, wl.c_std, (n_out, n_in, wl.g + wl.k))
        layers.append({"wb": wb, "ws": np.ones((n_out, n_in)), "c": c, "g": wl.g, "k": wl.k})
    return layers


def inputs(wl: Workload, n, seed=SEED_INPUTS, stream=0):
    """n raster-scanned input vectors of the workload's first-layer width."""
    r = _rng(seed, stream)
    n_in = wl.shape[0]
    if wl.input_kind == "uniform_pm1":
        return r.uniform(-1.0, 1.0, (n, n_in))
    if wl.input_kind == "pixels255":
        return np.round(r.uniform(0.0, 1.0, (n, n_in)) * 255.0) / 255.0
    if wl.input_kind == "pixels":
        return r.uniform(0.0, 1.0, (n, n_in))
    raise ValueError(wl.input_kind)


def calibration_inputs(wl: Workload, n=4096):
    return inputs(wl, n, seed=SEED_CALIB)


def poisson_arrivals(rate, n, seed=SEED_ARRIVALS):
    """arrival times (s) of n requests at `rate` per second."""
    r = _rng(seed, 0)
    return np.cumsum(r.exponential(1.0 / rate, n))


def request_mix(n, names, probs, seed=SEED_ARRIVALS):
    r = _rng(seed, 1)
    return [names[i] for i in r.choice(len(names), size=n, p=probs)]
