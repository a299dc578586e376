"""Atom types and term presets (oracle side).

Type table (reading): the paper types atoms through OpenBabel features that
only feed the learned term (Methods, "Scoring functions"); the physics terms
need only a van der Waals radius per atom and donor/acceptor flags
(definitions of E_long, E_clash, E_Hbond).  We use 8 types with X-Score /
Vina-style radii in Angstrom.
"""
import math

TYPE_NAMES = ("C_H", "C_P", "N_P", "N_D", "N_A", "O_A", "O_DA", "Cl_H")
#                 R     hydrophobic donor acceptor
TYPE_TABLE = (
    (1.9, True, False, False),   # C_H  carbon bonded only to C
    (1.9, False, False, False),  # C_P  carbon bonded to N or O
    (1.8, False, False, False),  # N_P  tertiary N, no H
    (1.8, False, True, False),   # N_D  N carrying H (donor)
    (1.8, False, False, True),   # N_A  N without H, <= 2 heavy neighbours
    (1.7, False, False, True),   # O_A  O without H
    (1.7, False, True, True),    # O_DA O carrying H
    (1.8, True, False, False),   # Cl_H
)
N_TYPES = 8


def radius(t):
    return TYPE_TABLE[t][0]


def hydrophobic(t):
    return TYPE_TABLE[t][1]


def donor(t):
    return TYPE_TABLE[t][2]


def acceptor(t):
    return TYPE_TABLE[t][3]


def hbond_pair(ti, tj):
    """Donor/acceptor pair in either direction (Methods, E_clash / E_Hbond)."""
    return (donor(ti) and acceptor(tj)) or (acceptor(ti) and donor(tj))


PRESET_TRIDS = 0
PRESET_VINA = 1

# TRIDS physics preset: E_long, E_clash, E_Hbond with the paper's weights
# w_long = 0.2, w_clash = 10, w_Hbond = 0.6 (Methods, E_dock; Table S4).
TRIDS_TERMS = ("long", "clash", "hbond")
TRIDS_WEIGHTS = (0.2, 10.0, 0.6)
TRIDS_LONG_DMAX = 10.0          # d_max of E_long
TRIDS_LONG_MU = 3.0             # Vina gauss2 offset on the surface distance
TRIDS_LONG_2SIG2 = 4.0          # Vina gauss2 width 2 A -> 2 sigma^2 = 4
TRIDS_HB_MU = 2.88              # E_Hbond mu
TRIDS_HB_SIGMA = 0.3            # E_Hbond sigma
TRIDS_HB_DMAX = 3.4             # E_Hbond d_Hmax
TRIDS_CLASH_DHB = 2.6           # d_clash for a donor/acceptor pair
CLASH_DMIN = 0.1                # floor of d inside log (reading: d -> 0 guard)

# Vina-form preset (five terms of the Vina function the paper builds on).
VINA_TERMS = ("gauss1", "gauss2", "repulsion", "hydrophobic", "hbond")
VINA_WEIGHTS = (-0.0356, -0.00516, 0.840, -0.0351, -0.587)
VINA_CUTOFF = 8.0

OUT_OF_GRID_K = 10.0            # penalty per Angstrom outside the map box

# Sampler constants (Methods, "Conformation sampling").
MC_BETA = 0.069
ADAM_LR = 0.1
ADAM_B1 = 0.9
ADAM_B2 = 0.999
ADAM_EPS = 1e-8
W_TOR = 0.01
TWO_PI = 2.0 * math.pi


def n_terms(preset):
    return 3 if preset == PRESET_TRIDS else 5


def default_weights(preset):
    return TRIDS_WEIGHTS if preset == PRESET_TRIDS else VINA_WEIGHTS


def term_cutoffs(preset, ti, tj):
    """Per-term hard cutoff distance for a (ti, tj) pair, or None = no term.

    A term contributes only while d < cutoff.  For clash the cutoff is d_clash
    (reading: the indicator is d < d_clash, which keeps the penalty
    continuous); for the hydrogen-bond terms a non donor/acceptor pair has no
    term at all.
    """
    rsum = radius(ti) + radius(tj)
    hb = hbond_pair(ti, tj)
    if preset == PRESET_TRIDS:
        dclash = TRIDS_CLASH_DHB if hb else rsum
        return (TRIDS_LONG_DMAX, dclash, TRIDS_HB_DMAX if hb else None)
    hyd = hydrophobic(ti) and hydrophobic(tj)
    c = VINA_CUTOFF
    return (c, c, c, c if hyd else None, c if hb else None)
