"""FP64 CPU oracle of the harmonic-basis 3PCF estimator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this directory.  The GPU
library never uses it, and it shares no code, header, table or helper with the GPU
library: both consume the seeded inputs of the ``synth`` package and nothing else.

Contents
--------
ref.py          plain NumPy estimator (direct trigonometry), for catalogues up to ~1e5 points
brute.py        brute-force triplet sum that needs no reference direction (tiny inputs)
hist.py         angular-histogram + Fourier-sum estimator (the histogram picture of the
                complexity discussion; each pair at its angular bin's centre)
fftlog.py       FFTLog chain of the modelling appendix (c_m, Gamma-ratio Hankel factors,
                A_{s1 s2} quadrature, I = U A V^T) for the functions A_0, A_1, A_2
oracle_cpu.c    plain C + OpenMP FP64 estimator with its own cube-grid search (large inputs)
cpu.py          ctypes wrapper of the compiled oracle_cpu.c
build.py        compiles oracle_cpu.c with gcc (-O2 -ffp-contract=off -fopenmp)

What the oracle computes (paper: harmonic-decomposition section, eqs. Xmdef,
zetaisohom, ubEstimator, eq_zeta_harmonic; binned estimator eqs. Xm.binned, zetamEst,
Ym/Zm.binned, zetamEst2); where the paper is silent or inconsistent, the steps below
state the reading taken (exponent sign exp(-i m phi), per-bin normaliser W_{p,b},
half-open chord-squared bins, bearing from local north through east):

1. pair geometry: delta = r_j - r_p, d2 = (dx*dx + dy*dy) + dz*dz in FP64, every
   operation rounded separately (no fused multiply-add);  pair kept iff
   E_0 <= d2 < E_nb; its bin is the b with E_b <= d2 < E_{b+1};
2. bearing: phi = atan2(delta . e_E, delta . e_N), position angle from local north
   through east, e_N = normalise(z - z_p r_p) (x-axis fallback at the poles),
   e_E = e_N x r_p;
3. multipoles: a_{m,b}(p) = sum_{j in b} w_j x_j exp(-i m phi_pj),
   W_{p,b} = sum_{j in b} w_j,  N_{p,b} = #{j in b};
4. normalise: X_m(b; p) = a_{m,b}(p) / W_{p,b}, and 0 where W_{p,b} = 0;
5. contract: zeta_m(b1, b2) = (1 / sum_p w_p) sum_p w_p x_p X_m(b1; p) conj(X_m(b2; p)),
   over all pivots, keeping the j = k terms;
   optionally without them (the diagonal overcount that the paper flags in the
   kappa^3 multipole-signal subsection): each pivot's product X(b) conj X(b) holds the
   terms k = j, sum_{j in b} (w_j x_j / W_{p,b})^2 for every m, which are then
   subtracted; brute.py drops them from the triplet sum directly (k != j);
   multi-field form (remark after eq. ubEstimator): the pivot carries field A, X(b1) is
   taken from field B and X(b2) from field C; optionally summed over the cyclic
   permutations of (A, B, C);
   pivots on a plane (positions [2, n], d2 = dx*dx + dy*dy, phi = atan2(dx, dy) from +y
   towards +x) use the same steps 3-5;
6. resum: zeta(b1, b2, phi) = sum_{m=-M}^{M} zeta_m exp(i m phi), zeta_{-m} = conj(zeta_m).

Parity of every function here is pinned by tests that do not re-type its formulas
(see tests/test_oracle_*.py): a closed-form three-point configuration, brute-force
triplets, exact invariants, the m = 0 annulus-mean identity, the Dirichlet-kernel
identity of the resummation, and brute-force pair counts.
"""
