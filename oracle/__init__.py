"""FP64 CPU oracle for the network-dynamics hot path (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package.  It shares no code with the HIP library.
"""
