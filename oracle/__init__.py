"""CPU oracle for the MFS elastance / mobility solve -- TEST INFRASTRUCTURE ONLY.

Importable only from tests/, __graft_entry__.smoke() and the CPU-baseline leg
of bench.py.  The GPU library never uses anything in this folder."""
