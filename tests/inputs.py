"""Seeded synthetic inputs shared by the oracle tests and the GPU parity
tests.  Holds none of the method's arithmetic: only grid sizes, potential
parameters, energies and counter-based random draws (splitmix64)."""
import math

MASK = (1 << 64) - 1


def splitmix64(state: int):
    """One step of splitmix64 (Steele, Lea, Flood 2014): returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return state, z ^ (z >> 31)


def uniforms(seed: int, n: int):
    """n doubles in [0, 1) from splitmix64, u = (x >> 11) * 2^-53."""
    out, s = [], seed
    for _ in range(n):
        s, x = splitmix64(s)
        out.append((x >> 11) * 2.0 ** -53)
    return out


SEED = 1508074410

# Rank-1 Yamaguchi pair potential: beta = 1, pair bound state at -0.1.
YAM_BETA = 1.0
YAM_KAPPA = math.sqrt(0.1)
YAM_LAMBDA = -4.0 * YAM_BETA * (YAM_BETA + YAM_KAPPA) ** 2 / math.pi

# Two-range attractive Yukawa sum, ranges 1 and 2 (equal weights).
YUK_RANGES = (1.0, 2.0)

# Small configuration (s-wave, 40 x 40 bins, cutoffs 10, 8 Gauss points per
# q bin, 16 on the cosine interval, E = 0.5).
C1 = dict(n_p=40, n_q=40, p_max=10.0, q_max=10.0, n_gq=8, n_gx=16, energies=(0.5,))
# Bench configuration (s-wave Yukawa sum, 150 x 150 bins, 20-point cosine
# rule, 8 energies spanning below and above breakup).
C2 = dict(n_p=150, n_q=150, p_max=10.0, q_max=10.0, n_gq=8, n_gx=20,
          energies=(-0.08, -0.05, -0.02, 0.05, 0.2, 0.5, 1.0, 2.0))
# Toy grid for single-element checks.
TOY_P = (0.0, 0.4, 0.9, 1.5, 2.2)
TOY_Q = (0.0, 0.5, 1.0, 1.6, 2.3)


def mlp_case(seed: int, nin: int, nh: int, nout: int, batch: int):
    """Parameters [W1 b1 .. W4 b4] (Glorot-uniform weights, small biases),
    inputs in [-2, 2) and targets in [-1, 1) for a 3-hidden-layer network."""
    dims = [(nh, nin), (nh, nh), (nh, nh), (nout, nh)]
    n_par = sum(o * i + o for o, i in dims)
    u = uniforms(seed, n_par + batch * (nin + nout))
    params, k = [], 0
    for o, i in dims:
        a = math.sqrt(6.0 / (o + i))
        params += [(2.0 * x - 1.0) * a for x in u[k:k + o * i]]
        k += o * i
        params += [0.1 * (2.0 * x - 1.0) for x in u[k:k + o]]
        k += o
    X = [4.0 * x - 2.0 for x in u[k:k + batch * nin]]
    k += batch * nin
    T = [2.0 * x - 1.0 for x in u[k:k + batch * nout]]
    return dims, params, X, T


def learn_draws(seed: int, n_var: int, n_mult: int, n_E: int, e_lo: float, e_hi: float):
    """Potential multipliers U[0.8, 1.2] (n_mult per variant, drawn first)
    and energies U[e_lo, e_hi] (n_E per variant), variant by variant."""
    u = uniforms(seed, n_var * (n_mult + n_E))
    mult, E = [], []
    for v in range(n_var):
        row = u[v * (n_mult + n_E):(v + 1) * (n_mult + n_E)]
        mult.append([0.8 + 0.4 * x for x in row[:n_mult]])
        E.append([e_lo + (e_hi - e_lo) * x for x in row[n_mult:]])
    return mult, E

# Three nucleons, pair s-waves (Sec. III.B eq.(gal) with spin and isospin):
# channels (pair spin s, pair isospin t) with the deuteron channel first;
# the 1S0 pair potential is the fitted Yukawa sum with both strengths times
# NUC_SINGLET_MULT (no bound pair), the 3S1 one the fitted sum itself.
NUC_DOUBLET = [(1, 0), (0, 1)]   # three-body spin 1/2
NUC_QUARTET = [(1, 0)]           # three-body spin 3/2
NUC_SINGLET_MULT = (0.7, 0.7)
