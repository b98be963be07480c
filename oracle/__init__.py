"""CPU oracle for Pi_MatMul.  TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check
and the benchmark's CPU-baseline leg; never by the library or its binding."""
