"""CPU oracle for the SNP-with-delays step.  Test infrastructure only: imported
by the test-suite, the smoke check and the CPU-baseline leg of the benchmark,
never by the product path."""
