"""CPU oracle for context-free path querying under relational semantics.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this package; only the test-suite, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the GPU path: the only common input is the
seeded generator package ``workloads``, which holds no query arithmetic.

Contents and what each follows:

* ``worklist`` (C, ``cfpq_worklist.c``): the least set of triples (A, i, j)
  containing the edge-derived triples and closed under every rule A -> B C,
  i.e. the relations R_A of section 2, which Theorem 2 says the matrix closure
  computes.  The main oracle.
* ``alg1``: Algorithm 1 of section 4.2 written out with numpy, one Boolean
  product per binary rule (Valiant's remark, section 3); gives the loop count
  of the paper's simultaneous update, and Valiant's closure a^+ of section 2
  truncated at a path length.
* ``brute``: CYK over a CNF grammar and enumeration of every path up to a
  length bound, straight from the definition of R_A (section 2).
* ``conjunctive``: Algorithm 1 generalised to conjunctive grammars (the
  conclusion's remark): T_A gains the AND over a rule's conjuncts of their
  products; ``brute.conj_cyk_table`` is CYK for such grammars.
* ``single_path``: the path lengths of section 5 (l_A = l_B + l_C when a step
  first adds A to a cell, kept afterwards; the smallest sum when one step
  offers several) and a witness path for any stored length.

Pins (tests/test_oracle_*.py): the worked example of section 4.3 (every
printed T_k, the loop count 6 and all seven R_A), a closed form for two label
cycles of coprime length, textbook special cases (transitive closure, CYK on a
chain, bracket matching, terminal-only grammars), brute force on tiny graphs,
and invariants (closure, monotonicity, permutation equivariance, disjoint
union); for the lengths, breadth-first search, chains, the two-cycle closed
form, a first-found-is-kept case and CYK on every witness; for the language
enumeration ``brute.cfg_words``, languages known in closed form (a^n b^n,
balanced words with their Catalan counts, equal letter counts, palindromes, a
unit cycle through nullable symbols); for ``brute.conj_paths_up_to``, Boolean
matrix powers (a path spells a^n b^n c^n iff it is in M_a^n M_b^n M_c^n).
Every function here has at least one such pin, and mutation harnesses check
that planted mistakes break one.
"""
