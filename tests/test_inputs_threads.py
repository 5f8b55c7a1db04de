"""The input generator's Delaunay builder keeps its working state per
thread: workloads built on several host threads at once (as the pipelined
server prepares jobs) equal the same workloads built one after another."""
import threading

import numpy as np

import qm_inputs as qi


def test_concurrent_builds_equal_sequential_ones():
    makers = [lambda i=i: qi.uniform_cube(800 + 97 * i, seed=i, B=2.0, spheres=(0.3,)) for i in range(6)]
    ref = [m() for m in makers]
    got = [None] * len(makers)

    def run(k):
        got[k] = makers[k]()

    th = [threading.Thread(target=run, args=(k,)) for k in range(len(makers))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for a, b in zip(got, ref):
        assert np.array_equal(a.xyz, b.xyz) and np.array_equal(a.tets, b.tets) and np.array_equal(a.adj, b.adj)
