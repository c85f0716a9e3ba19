"""CPU oracle for restarted GMRES and the learned preconditioner: test infrastructure only.

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import this package.  It shares no code with the GPU library.
"""
