"""CPU oracle for the Monte Carlo NEGF hot path (FP64, plain and slow on purpose).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import, call, link or execute anything in this package.  The HIP library never calls
it, and it shares no code, headers, tables or helpers with the HIP path.

Contents:
  dense.py    dense direct NEGF + elastic Buttiker solve: lead self-energies, G^r,
              terminal transmissions, the probe-conservation system, the lead current,
              the walker's transition kernel and its exact absorption probabilities,
              and Vose's alias tables.
  walker.c    a plain C random walker on the same Philox4x32-10 streams as the GPU
              (the paper's cumulative-sum sampler, or an alias table given to it).
  walker.py   ctypes wrapper and build step for walker.c.
  grad.py     dI/dV_i and dI/dgamma_i of the DIRECT current: reverse-mode differentiation
              (torch autograd, CPU) of a dense evaluation, and central differences.
  columns.py  sampled columns of G at sizes the dense solve cannot hold (sparse LU).
  interp.py   step-6' rows interpolated between energy nodes (Sec. V A, "Interpolation").
  weighted.py importance-sampled walks and their path-ratio estimator (Sec. V A,
              "Improved estimator").
  score.py    score-function gradient of the Monte Carlo estimator and expected counts.
  inelastic.py  step 7' (Sec. II F): the energy draw of inelastic Buttiker walks, its
              threshold table, the exact exit distribution of the (energy, probe) chain and
              the energy-resolved current; walks by walker.c.
"""
