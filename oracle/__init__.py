"""CPU oracle for the l1-regularised log-det estimator — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct float64 code that states what the GPU library
computes, written from the paper (Treister, Turek, Yavneh, "A multilevel
framework for sparse optimization with application to inverse covariance
estimation and logistic regression"). Only ``tests/``, the package smoke check
(``__graft_entry__.smoke``) and the benchmark's CPU-baseline leg may import it;
the GPU library and its Python binding never import, link or execute anything
here, and this package never imports the library.

Modules
  core        objective, gradient, KKT measure, free set (Sections 3, 4, 5)
  quic_plain  solution oracle: dense proximal Newton on the full free set
  steps       per-step definitions of one block update (Section 6, App. A)
  mlbcd       the multilevel cycle over block relaxations (Alg. 1, Alg. 2, Sec. 7)
  bruteforce  support enumeration for n <= 4 (independent pin)
  cd          ctypes wrapper of the plain C coordinate-descent loop
"""
