"""CPU oracle for the Flood-complex flooding path -- TEST INFRASTRUCTURE.

A plain, slow, obviously correct implementation of what the GPU path
computes, written from the paper's definitions:

* ``fps``        farthest-point landmarks (greedy k-centre), float32 recipe
* ``delaunay``   Delaunay triangulation of the landmarks: brute-force empty
                 sphere on tiny inputs, a local-Delaunay certificate for any
                 size, exact predicates (FP64 filter + exact rationals)
* ``flood``      the sampled flood values f_P (Def. 1, Sec. 4.1, Lemma 6)
                 in FP64, brute or Lemma-7 masked; closure; winners and the
                 analytic gradient; the exact covering radius r_exact on tiny
                 inputs; the grid covering radius h of Lemma 6
* ``ph``         Z/2 persistence by column reduction and bottleneck matching

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library and
must never be reached from the product path.
"""
