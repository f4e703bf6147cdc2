"""FP64 CPU oracle (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this
package.  It shares no code with the HIP library or its binding.
"""
