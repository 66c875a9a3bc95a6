"""Client process for the multi-process tests: attaches to a context another
process shared and runs the life-cycle calls it reads on stdin, one JSON
reply per line on stdout.  Not a test module itself."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    from paper_1712_04495_amd import cosched as cs
    rc, ctx = cs.sched_attach(sys.argv[1])
    print(json.dumps({"rc": rc, "pid": os.getpid()}), flush=True)
    if rc != 0:
        return 1
    for line in sys.stdin:
        op, *args = line.split()
        a = [int(x) for x in args]
        if op == "register":
            rc, j = cs.sched_register(ctx, a[0], a[1])
            out = {"rc": rc, "job": j}
        elif op == "admit":
            out = {"rc": cs.sched_admit(ctx, a[0], 0, a[1], a[2])}
        elif op == "wait":
            out = {"rc": cs.sched_wait(ctx, a[0], a[1])}
        elif op == "release":
            out = {"rc": cs.sched_release(ctx, a[0], -1, a[1])}
        elif op == "own":
            out = {"rc": cs.sched_set_owner(ctx, a[0], os.getpid())}
        elif op == "reservation":
            rc, v = cs.sched_reservation(ctx, a[0])
            out = {"rc": rc, "res": v}
        elif op == "stats":
            rc, st = cs.sched_stats(ctx)
            out = {"rc": rc, **st}
        elif op == "quit":
            out = {"rc": cs.sched_destroy(ctx)}
            print(json.dumps(out), flush=True)
            return 0
        else:
            out = {"rc": -99}
        print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
