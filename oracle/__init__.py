"""FP64 CPU oracle for the low-scaling GW path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path:
it reads the seeded inputs from ``gwinputs`` and nothing else.

Convention (the paper prints i-factors that would make chi and Sigma purely
imaginary; the real form below is the same physics without them):

* eps_bar = eps - mu_F, mu_F = (eps_HOMO + eps_LUMO) / 2
* D^occ(tau) = sum_{i occ} exp(+eps_bar_i tau) c_i c_i^T,
  D^vir(tau) = sum_{a vir} exp(-eps_bar_a tau) c_a c_a^T   (Eq. 2, tau >= 0)
* chi_PQ(tau) = - sum_{mu sigma} [sum_lambda (lambda sigma P) D^occ_{mu lambda}]
                                 [sum_nu (mu nu Q) D^vir_{nu sigma}]      (Eq. 3)
  per spin channel; the closed-shell spin factor s = 2 enters the
  screening step.
* chi(i w_k) = 2 s sum_j c_kj chi(tau_j); eps = 1 - L^T chi L; V = L L^T;
  W^c = L (eps^-1 - 1) L^T; W^c(tau_j) = 1/2 sum_k d_jk W^c(i w_k)  (Eqs. 5-9)
* B^n_{mu P} = sum_nu C_{n nu} (nu mu P); Sigma^occ_n(tau) =
  <D^occ(tau), B^n W^c(tau) B^nT>_F, Sigma^vir_n likewise with D^vir;
  Sigma^x_n = -<D^occ(0), B^n V B^nT>_F                             (Eqs. 10-11)
* Sigma^c_n(i w_k) = sum_j c_kj (S^vir - S^occ)(tau_j)
                     + i sum_j s_kj (S^vir + S^occ)(tau_j)
* Thiele continued-fraction Pade on the i w nodes and Newton on Eq. 12.

Parity status per function is stated in each module's header.
"""
