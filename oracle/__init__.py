"""Plain, slow FP64 CPU oracle for self-learning determinantal QMC.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under ``oracle/``; only the tests, the smoke check and the
CPU-baseline leg of the benchmark do.  The oracle shares no code with the HIP
path: it is written from the paper (Xu, Qi, Liu, Fu, Meng, "Self-Learning
Determinantal Quantum Monte Carlo Method", arXiv:1612.03804) and from the
textbook definitions it relies on, in NumPy/SciPy FP64, with no blocking,
fusion or reordering beyond what those definitions state.

Modules
    philox     counter-based generator Philox4x64-10 (Salmon et al., SC'11)
    lattice    hopping matrix, slice matrices, chain product, direct det / G,
               space-time block matrix              (Basics of DQMC, Eq. 1)
    stable     QR/UDV-stabilised log|det|, sign and G
    fock       brute-force many-body trace for tiny lattices
    dqmc       local-update sweep: determinant ratio, rank-1 G update, wrap,
               periodic recompute                   (Basics of DQMC)
    effective  effective action, its single-flip change, colour classes,
               effective sweep and cumulative update (Eqs. 2 and 4)
    fit        multi-linear regression and R^2      (Eq. 3, Results)
    autocorr   autocorrelation function and integrated time (Fig. 1 caption)
    checkerboard  sparse (checkerboard) split of the kinetic factor and the
               weight and G built on it             (Formalism of SLDQMC)
    measure    equal-time observables from G, time-displaced G, Ising
               susceptibility                       (Basics of DQMC, Results)
    net        convolutional correction to the effective action, its
               gradient and Adam                    (Formalism of SLDQMC, Eq. 2)
    bilayer    the four-flavour bilayer weight with the bare Ising action
               and its local sweep                  (Results, Eq. 6)

Every function says which passage it follows.  Parity of the physics-level
numbers of the paper (autocorrelation times of its bilayer model at its
parameters, critical exponents) is unpinned: they need couplings the paper
does not state and production runs; the bilayer module reproduces the
method's comparison at small sizes, not those numbers.
"""
