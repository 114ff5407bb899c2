"""Plain CPU float64 oracle for circuit-cutting reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing in the library calls this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark import
it.  It shares no code with the HIP path: it takes the same seeded inputs
(from ``workloads``) and computes the result from the definitions in the
paper, slowly and in the most direct form.

Modules
  pauli        measured subcircuit variants -> Pauli-basis tensors (Sec. II-A)
  reconstruct  brute-force sum over all 4^K cut assignments (Eq. (1)) and
               per-entry variable elimination (the same multilinear sum)
  outputs      top-k and marginals of a probability vector (Eq. (10))
  plancost     multiplication count of a contraction sequence (Sec. III-C)
  mlp          float64 MLP forward/backward for the learned cost model
  hss          heavy state selection (Alg. 1) and its metrics (Eqs. (9)-(13))
  cutfind      greedy graph growing cut search (Alg. 2-3, Table I), Eq. (6)
"""
