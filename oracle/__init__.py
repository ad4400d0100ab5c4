"""CPU oracle for the dynamic-data-rate actor method.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  The HIP library never calls it and shares no code with it.

It is a plain sequential dataflow scheduler that fires one actor at a time
(the firing rule of Sec. 2.2), with FP64 arithmetic for the predistortion
network and exact integer arithmetic for motion detection.  Batched GPU firing
is a different schedule of the same firings; by the single-writer /
single-reader FIFO channels and blocking reads of Sec. 2.2 / 3.2 (Kahn
determinacy) both must produce identical token streams, so the plain
definition computed here is the expected result.

Modules:
    dataflow  FIFO channel, actor base class, scheduler (Sec. 2.2, 3.1)
    dpd       the predistortion network P -> FIR_b -> A (Sec. 4.2)
    motion    the motion-detection network Detect -> Gate (Sec. 4.1 idiom)
    md_paper  the paper's motion-detection pipeline Gauss -> Thres -> Med (Sec. 4.1)
    pa        memory-polynomial PA, Wirtinger adjoints, finite differences

Every function's docstring names the passage it follows.  Functions whose
result is not pinned by a test say "parity unpinned" (none at present).
"""
